"""Parity at the benchmark's sizes and launch configuration.

The headline workload (70,000 x 10,700, 9M training entries, K = 50, B = 32)
is stepped on the GPU with the schedule bench.py tunes, and single steps
(t = 0 and mid-run) are compared element by element with the FP64 oracle's
full step.  The dense spectrogram-shaped workload (1025 x 100,000, K = 64,
beta = 0.5, B = 16) and the large ratings workload (480,000 x 17,800, 90M
training entries, K = 100, B = 64) are checked the same way at their full
sizes and launch configurations (each oracle step takes about ten seconds);
smaller versions of both also run in seconds.  Each full-size workload also
runs its whole chain (1000 iterations, burn-in 500), and its held-out RMSE
is compared with the oracle's stored full run."""
import json
import os

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
        _FULL[name] = workloads.by_name(name)
    return _FULL[name]


def _stored_rmse(name):
    """The FP64 oracle's held-out RMSE after the workload's full run, written
    by tests/golden/make_heldout_rmse.py (which calls only the oracle)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "heldout_rmse.json")
    with open(path) as f:
        return json.load(f)[name]


def _long_run_rmse(s, wl, name):
    """Runs the whole chain from t = 0 and checks its held-out RMSE against
    the stored oracle value: within 1%, same T, burn-in and thinning."""
    ref = _stored_rmse(name)
    assert (ref["T"], ref["burn_in"], ref["thin"], ref["n_heldout"]) == (wl.T, wl.burn_in, wl.thin, len(wl.hval))
    s.step(wl.T, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    g = s.heldout_rmse()
    assert s.num_samples() == ref["n_kept"]
    assert abs(g - ref["heldout_rmse"]) <= 0.01 * ref["heldout_rmse"], (g, ref["heldout_rmse"])
    return g


def test_sparse_ratings_70k_1000_iterations_rmse_parity():
    """70,000 x 10,700 (9M training entries, K = 50, B = 32) with the tuned
    schedule the benchmark uses: 1000 iterations (burn-in 500, moments every
    10th), held-out RMSE within 1% of the oracle's full run."""
    wl = _full("sparse_ratings_70k")
    s = pkg.PSGLD.from_workload(wl)
    s.tune(wl.eps_a, wl.eps_t0, wl.eps_gamma, candidates=(16, 32, 64, 128), iters=wl.B)
    _long_run_rmse(s, wl, "sparse_ratings_70k")
    s.close()
    _FULL.pop("sparse_ratings_70k")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("bf16", [False, True])
def test_dense_tweedie_full_size_step_parity(bf16):
    """1025 x 100,000 with the benchmark's options (blocks of 6,250 columns on
    the dense kernels), single steps at t = 0 and t = 3."""
    wl = _full("dense_tweedie_1025x100k")
    prec = pkg.PSGLD_BF16_DENSE if bf16 else pkg.PSGLD_FP32
    s = pkg.PSGLD.from_workload(wl, dense=True, precision=prec)
    err0, _ = step_parity(wl, 0, sampler=s)
    err1, _ = step_parity(wl, 2, sampler=s)
    s.close()
    tol = TOL_BF16 if bf16 else TOL_FP32
    assert err0 <= tol and err1 <= tol, (err0, err1)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["f32", "bf16", "bf16v"])
def test_dense_tweedie_1000_iterations_rmse_parity(precision):
    """The same workload's full run on the dense kernels with FP32 operands,
    BF16 operands, and BF16 operands on BF16-stored values: held-out RMSE
    within 1% of the oracle's (FP64, FP32 values) full run, so the BF16
    paths reach the plain FP32 result."""
    wl = _full("dense_tweedie_1025x100k")
    prec = {"f32": pkg.PSGLD_FP32, "bf16": pkg.PSGLD_BF16_DENSE, "bf16v": pkg.PSGLD_BF16_DENSE_VALUES}[precision]
    s = pkg.PSGLD.from_workload(wl, dense=True, precision=prec)
    _long_run_rmse(s, wl, "dense_tweedie_1025x100k")
    s.close()
    if precision == "bf16v":
        _FULL.pop("dense_tweedie_1025x100k")


@pytest.mark.timeout(600)
def test_large_ratings_full_size():
    """480,000 x 17,800 (90M training entries, K = 100, B = 64) with the
    schedule the benchmark tunes: single steps at t = 0 and mid-run (t = 9,
    another part, element by element against the oracle's full step), then
    the whole 1000-iteration run, whose held-out RMSE is within 1% of the
    oracle's full run."""
    wl = _full("sparse_ratings_480k")
    s = pkg.PSGLD.from_workload(wl)
    s.tune(wl.eps_a, wl.eps_t0, wl.eps_gamma, candidates=(16, 32, 64, 128), iters=wl.B)
    state0 = s.get_state()
    err0, _ = step_parity(wl, 0, sampler=s)
    err1, _ = step_parity(wl, 8, sampler=s)
    assert err0 <= TOL_FP32 and err1 <= TOL_FP32, (err0, err1)
    s.set_state(state0)
    _long_run_rmse(s, wl, "sparse_ratings_480k")
    s.close()
    _FULL.pop("sparse_ratings_480k")
