"""psgld_step_static, the entry point for callers that cannot allocate: the
same iterations as psgld_step with the kernels' scratch (split-share
partials, arrival counters, step sizes) in one static device array per GPU.
Checked through the C ABI against psgld_step on an identical context,
bitwise, on two calls in a row, the second on a smaller input; every device
allocation of the contexts goes through counting hooks, which must see no
call during the allocation-free steps."""
import numpy as np
import pytest

import paper_1506_01418_amd as pkg
import workloads
from test_gpu_dense import dense_case

pytestmark = pytest.mark.gpu


def _outputs(s):
    return (*s.factors(), *s.posterior_mean(), *s.posterior_var(), s.heldout_predictions(),
            np.array([s.num_samples(), s.iteration()]))


def _pair(wl, epg):
    """(regular, static) contexts of one workload, allocating through
    counting hooks, with the same fixed schedule."""
    out = []
    for _ in range(2):
        s = pkg.PSGLD.from_workload(wl, allocator=pkg.TorchAllocator(0, 0))
        s.tune(wl.eps_a, wl.eps_t0, wl.eps_gamma, candidates=(epg,))
        out.append(s)
    return out


def _static_step(s, wl, n):
    calls = s.allocator.calls
    pkg.psgld_step_static(s.ctx, n, pkg.psgld_eps_schedule(wl.eps_a, wl.eps_t0, wl.eps_gamma))
    s.sync()
    assert s.allocator.calls == calls          # no device allocation in the call


def test_static_step_matches_psgld_step_on_two_calls():
    big = workloads.sparse_ratings(I=60_000, J=2_000, nnz=3_000_000, K_true=30, K=100, B=4, zipf_a=1.1,
                                   data_seed=1104, chain_seed=2104, name="skewed_60k")
    big.burn_in, big.thin = 10, 3
    ref, st = _pair(big, 16)                   # many split shares per head column
    ref.step(25, big.eps_a, big.eps_t0, big.eps_gamma)
    _static_step(st, big, 25)
    for a, b in zip(_outputs(ref), _outputs(st)):
        assert np.array_equal(a, b, equal_nan=True)
    # second call: a smaller input on a fresh pair of contexts, then the
    # first pair again, to show the shared scratch holds nothing over
    small = workloads.random_sparse(900, 500, 30_000, 16, 6, beta=2.0, phi=0.5, zipf_a=1.0,
                                    data_seed=93, chain_seed=94, burn_in=4, thin=2)
    ref2, st2 = _pair(small, 16)
    ref2.step(9, small.eps_a, small.eps_t0, small.eps_gamma)
    _static_step(st2, small, 9)
    for a, b in zip(_outputs(ref2), _outputs(st2)):
        assert np.array_equal(a, b, equal_nan=True)
    ref.step(7, big.eps_a, big.eps_t0, big.eps_gamma)
    _static_step(st, big, 7)
    for a, b in zip(_outputs(ref), _outputs(st)):
        assert np.array_equal(a, b, equal_nan=True)
    for s in (ref, st, ref2, st2):
        s.close()


def test_static_step_rejects_what_it_cannot_run():
    wl = workloads.random_sparse(300, 220, 6000, 12, 4, data_seed=95, chain_seed=96)
    s = pkg.PSGLD.from_workload(wl)
    sched = pkg.psgld_eps_schedule(wl.eps_a, wl.eps_t0, wl.eps_gamma)
    with pytest.raises(pkg.PsgldError) as e:
        pkg.psgld_step_static(s.ctx, 65537, sched)
    assert e.value.status == pkg.PSGLD_E_ARG
    s.close()
    d = dense_case(128, 600, 16, 2, 0.5, density=0.9, seed=97)
    s = pkg.PSGLD.from_workload(d, dense=True, dense_min_cols=1)
    with pytest.raises(pkg.PsgldError) as e:
        pkg.psgld_step_static(s.ctx, 3, sched)
    assert e.value.status == pkg.PSGLD_E_UNSUPPORTED
    s.close()
