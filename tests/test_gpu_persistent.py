"""Persistent stepping (options.persistent): iterations run in cooperative
single launches with a grid-wide barrier between iterations, for one
context or for a batch of contexts.  Results must be bitwise those of one
launch per iteration, across call lengths (including more iterations than
one launch takes), burn-in, thinning and held-out sums, and contexts with
dense blocks keep their per-iteration launches."""
import numpy as np
import pytest

import paper_1506_01418_amd as pkg
import workloads
from parity import TOL_FP32, step_parity
from test_gpu_dense import dense_case

pytestmark = pytest.mark.gpu


def _outputs(s):
    return (*s.factors(), *s.posterior_mean(), *s.posterior_var(), s.heldout_predictions(),
            np.array([s.num_samples(), s.iteration()]))


def _assert_same(a, b):
    for x, y in zip(_outputs(a), _outputs(b)):
        assert np.array_equal(x, y, equal_nan=True)


CASES = {
    "K5_gamma": lambda: workloads.random_sparse(301, 199, 9000, 5, 3, beta=0.0, prior="exponential",
                                                mirror=True, data_seed=71, chain_seed=72),
    "K16_gauss": lambda: workloads.random_sparse(900, 500, 30_000, 16, 6, beta=2.0, phi=0.5, zipf_a=1.0,
                                                 data_seed=73, chain_seed=74),
    "K50_zipf": lambda: workloads.random_sparse(3000, 800, 150_000, 50, 4, beta=2.0, phi=0.5, zipf_a=1.0,
                                                data_seed=75, chain_seed=76),
    "K100_B8": lambda: workloads.random_sparse(1500, 1100, 80_000, 100, 8, beta=2.0, phi=0.4,
                                               data_seed=77, chain_seed=78),
    "K8_poisson": lambda: workloads.dense_poisson(),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_persistent_matches_single_launches(name):
    wl = CASES[name]()
    eager = pkg.PSGLD.from_workload(wl, burn_in=7, thin=3, graph_iters=-1)
    pers = pkg.PSGLD.from_workload(wl, burn_in=7, thin=3, persistent=1)
    for n in (3, 1, 40, 300, 9):          # 300 > one launch's 256 iterations
        eager.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        pers.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    _assert_same(eager, pers)
    eager.close()
    pers.close()


def test_persistent_batch_matches_alone():
    wls = [CASES[n]() for n in ("K5_gamma", "K16_gauss", "K50_zipf", "K8_poisson")]
    wls.append(dense_case(128, 300, 16, 2, 0.5, density=0.9, seed=79))
    dense = [False] * 4 + [True]
    alone = [pkg.PSGLD.from_workload(wl, dense=d, burn_in=5, graph_iters=-1, dense_min_cols=1)
             for wl, d in zip(wls, dense)]
    first = pkg.PSGLD.from_workload(wls[0], burn_in=5, persistent=1)
    together = [first] + [pkg.PSGLD.from_workload(wl, dense=d, burn_in=5, persistent=1, stream=first.stream(),
                                                  dense_min_cols=1)
                          for wl, d in zip(wls[1:], dense[1:])]
    scheds = [(wl.eps_a, wl.eps_t0, wl.eps_gamma) for wl in wls]
    for plan in ([12, 12, 7, 12, 12], [30, 0, 30, 5, 2]):
        for s, sc, n in zip(alone, scheds, plan):
            s.step(n, *sc)
        pkg.PSGLD.step_batch(together, plan, scheds)
    for a, b in zip(alone, together):
        _assert_same(a, b)
    for s in reversed(together):
        s.close()
    for s in alone:
        s.close()


def test_persistent_state_keeps_single_step_parity():
    wl = CASES["K50_zipf"]()
    s = pkg.PSGLD.from_workload(wl, persistent=1)
    err, s = step_parity(wl, 21, sampler=s)
    assert err <= TOL_FP32, err
    s.close()


def test_persistent_serving_matches_alone():
    wls = [CASES[n]() for n in ("K5_gamma", "K16_gauss", "K8_poisson")]
    for wl in wls:
        wl.burn_in, wl.thin = 10, 2
    srv = pkg.Server(hbm_budget=4 << 30, max_active=8, iters_per_tick=9, persistent=True)
    ids = [srv.submit(wl, 30) for wl in wls]
    for _ in range(100):
        running, queued, _ = srv.tick()
        if running == 0 and queued == 0:
            break
    for jid, wl in zip(ids, wls):
        assert srv.info(jid)["state"] == pkg.PSGLD_JOB_DONE, srv.error(jid)
        Wm, Hm, Wv, Hv, _ = srv.result(jid)
        s = pkg.PSGLD.from_workload(wl)
        s.step(30, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        for x, y in zip((Wm, Hm, Wv, Hv), (*s.posterior_mean(), *s.posterior_var())):
            assert np.array_equal(x, y)
        s.close()
    srv.close()


@pytest.mark.parametrize("grid", [1, 7])
def test_persistent_small_grid_matches_single_launches(grid):
    """Persistent launches with far fewer work-groups than tasks: each
    work-group runs many tasks of an iteration in turn, and the tasks of
    Zipf-skewed columns combine their groups' partial sums in LDS, which the
    next task of the same work-group reuses.  Bitwise equal to per-iteration
    launches."""
    wl = CASES["K50_zipf"]()
    eager = pkg.PSGLD.from_workload(wl, burn_in=5, thin=2, graph_iters=-1)
    pers = pkg.PSGLD.from_workload(wl, burn_in=5, thin=2, persistent=1, persistent_grid=grid)
    for n in (2, 19):
        eager.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        pers.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    _assert_same(eager, pers)
    eager.close()
    pers.close()
