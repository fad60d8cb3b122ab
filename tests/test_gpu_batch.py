"""Batched stepping (psgld_step_batch): contexts of one kernel variant share
one launch per iteration through a device job table.  Each context must
step to the same bits as psgld_step on it alone, and a batched step must
stay within the single-step parity bound against the oracle."""
import numpy as np
import pytest

import oracle
import paper_1506_01418_amd as pkg
import workloads
from parity import TOL_FP32, oracle_config, scaled_error
from test_gpu_dense import dense_case

pytestmark = pytest.mark.gpu


def _cases():
    return [
        workloads.random_sparse(400, 300, 9000, 8, 4, beta=1.0, prior="exponential", mirror=True,
                                data_seed=31, chain_seed=32),
        workloads.random_sparse(900, 500, 30_000, 16, 6, beta=2.0, phi=0.5, zipf_a=1.0,
                                data_seed=33, chain_seed=34),
        workloads.random_sparse(300, 650, 12_000, 16, 3, beta=2.0, data_seed=35, chain_seed=36),
        workloads.random_sparse(2000, 800, 60_000, 50, 8, beta=2.0, phi=0.4, zipf_a=1.0,
                                data_seed=37, chain_seed=38),
        workloads.random_sparse(150, 120, 3000, 5, 2, beta=0.0, prior="exponential", mirror=True,
                                data_seed=39, chain_seed=40),
    ]


def _outputs(s):
    return (*s.factors(), *s.posterior_mean(), *s.posterior_var(), s.heldout_predictions(),
            np.array([s.num_samples(), s.iteration()]))


def _shared(wls, dense_last=False, **kw):
    """Samplers on one stream (the first sampler's)."""
    first = pkg.PSGLD.from_workload(wls[0], **kw)
    out = [first]
    for m, wl in enumerate(wls[1:]):
        dense = dense_last and m == len(wls) - 2
        out.append(pkg.PSGLD.from_workload(wl, dense=dense, stream=first.stream(), dense_min_cols=1, **kw))
    return out


def _close(samplers):
    for s in reversed(samplers):
        s.close()


def _sched(wl):
    return (wl.eps_a, wl.eps_t0, wl.eps_gamma)


def test_batch_matches_each_context_alone():
    wls = _cases() + [dense_case(128, 300, 16, 2, 0.5, density=0.9, seed=41)]
    alone = [pkg.PSGLD.from_workload(wl, dense=(m == len(wls) - 1), burn_in=5, thin=2, dense_min_cols=1)
             for m, wl in enumerate(wls)]
    together = _shared(wls, dense_last=True, burn_in=5, thin=2)
    plans = [[12, 7, 12, 3, 12, 9], [1, 20, 0, 5, 8, 20]]
    for plan in plans:
        for s, wl, n in zip(alone, wls, plan):
            s.step(n, *_sched(wl))
        pkg.PSGLD.step_batch(together, plan, [_sched(wl) for wl in wls])
    for a, b in zip(alone, together):
        for x, y in zip(_outputs(a), _outputs(b)):
            assert np.array_equal(x, y, equal_nan=True)
    _close(together)
    for s in alone:
        s.close()


def test_batched_step_parity():
    wls = _cases()
    samplers = _shared(wls)
    pkg.PSGLD.step_batch(samplers, [6, 3, 9, 4, 6], [_sched(wl) for wl in wls])
    chains = []
    for s, wl in zip(samplers, wls):
        ch = oracle.Chain(oracle_config(wl), wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
        W, H = s.factors()
        ch.set_state(W, H, s.iteration())
        chains.append((ch, ch.run(1, bounds=True)))
    pkg.PSGLD.step_batch(samplers, [1] * len(wls), [_sched(wl) for wl in wls])
    for s, (ch, (bW, bH)) in zip(samplers, chains):
        W, H = s.factors()
        err = max(scaled_error(W, ch.W, bW).max(), scaled_error(H, ch.H, bH).max())
        assert err <= TOL_FP32, err
    _close(samplers)


def test_batch_rejects_bad_arguments():
    wls = _cases()[:2]
    a = pkg.PSGLD.from_workload(wls[0])
    b = pkg.PSGLD.from_workload(wls[1])            # its own stream
    with pytest.raises(pkg.PsgldError) as e:
        pkg.PSGLD.step_batch([a, b], [1, 1], [_sched(wls[0]), _sched(wls[1])])
    assert e.value.status == pkg.PSGLD_E_ARG
    with pytest.raises(pkg.PsgldError) as e:
        pkg.PSGLD.step_batch([a, a], [1, 1], [_sched(wls[0])] * 2)
    assert e.value.status == pkg.PSGLD_E_ARG
    assert a.iteration() == 0 and b.iteration() == 0
    b.close()
    a.close()
