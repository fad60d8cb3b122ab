"""Serving loop (psgld_server_*): FIFO admission under an HBM budget,
batched ticks, retirement.  A served job's posterior moments and held-out
RMSE must be bitwise those of the same run on a context of its own."""
import numpy as np
import pytest

import paper_1506_01418_amd as pkg
import workloads
from test_gpu_dense import dense_case

pytestmark = pytest.mark.gpu

N_ITER = 40


def _mix():
    wls = [
        workloads.random_sparse(400, 300, 9000, 8, 4, beta=1.0, prior="exponential", mirror=True,
                                data_seed=51, chain_seed=52),
        workloads.random_sparse(900, 500, 30_000, 16, 6, beta=2.0, phi=0.5, zipf_a=1.0,
                                data_seed=53, chain_seed=54),
        workloads.random_sparse(300, 650, 12_000, 16, 3, beta=2.0, data_seed=55, chain_seed=56),
        workloads.random_sparse(1200, 800, 50_000, 64, 8, beta=2.0, phi=0.4, zipf_a=1.0,
                                data_seed=57, chain_seed=58),
        dense_case(128, 300, 16, 2, 0.5, density=0.9, seed=59),
        workloads.random_sparse(150, 120, 3000, 32, 2, beta=1.0, prior="exponential", mirror=True,
                                data_seed=60, chain_seed=61),
    ]
    for wl in wls:
        wl.burn_in, wl.thin = 12, 2
    return wls


def _is_dense(wl):
    return wl.dense is not None


def _drain(srv, max_ticks=200):
    for _ in range(max_ticks):
        running, queued, _ = srv.tick()
        if running == 0 and queued == 0:
            return
    raise AssertionError("server did not drain")


def test_served_jobs_match_runs_alone():
    wls = _mix()
    srv = pkg.Server(hbm_budget=8 << 30, max_active=4, iters_per_tick=7)
    ids = [srv.submit(wl, N_ITER, dense=_is_dense(wl), dense_min_cols=1) for wl in wls]
    _drain(srv)
    for jid, wl in zip(ids, wls):
        assert srv.info(jid)["state"] == pkg.PSGLD_JOB_DONE, srv.error(jid)
        Wm, Hm, Wv, Hv, rmse = srv.result(jid)
        s = pkg.PSGLD.from_workload(wl, dense=_is_dense(wl), dense_min_cols=1)
        s.step(N_ITER, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        aWm, aHm = s.posterior_mean()
        aWv, aHv = s.posterior_var()
        for x, y in ((Wm, aWm), (Hm, aHm), (Wv, aWv), (Hv, aHv)):
            assert np.array_equal(x, y)
        assert rmse == s.heldout_rmse()
        s.close()
        srv.release(jid)
    srv.close()


def test_admission_respects_budget_and_order():
    wls = _mix()
    est = [pkg.psgld_server_estimate_bytes(pkg.psgld_job_from(wl, N_ITER, dense=_is_dense(wl))[0]) for wl in wls]
    budget = int(1.3 * max(est))
    srv = pkg.Server(hbm_budget=budget, max_active=8, iters_per_tick=10)
    ids = [srv.submit(wl, N_ITER, dense=_is_dense(wl)) for wl in wls]
    started = []
    for _ in range(200):
        running, queued, _ = srv.tick()
        infos = [srv.info(j) for j in ids]
        held = sum(i["bytes"] for i in infos if i["state"] == pkg.PSGLD_JOB_RUNNING)
        assert held <= budget
        for j, i in zip(ids, infos):
            if i["state"] != pkg.PSGLD_JOB_QUEUED and j not in started:
                started.append(j)
            if i["state"] == pkg.PSGLD_JOB_RUNNING:
                assert 0 < i["bytes"] <= i["est_bytes"]     # the estimate bounds the allocation
        if running == 0 and queued == 0:
            break
    assert started == ids                                    # FIFO admission
    assert all(srv.info(j)["state"] == pkg.PSGLD_JOB_DONE for j in ids)
    # a job larger than the whole budget is refused at submission
    small = pkg.Server(hbm_budget=min(est) // 2, max_active=2, iters_per_tick=5)
    with pytest.raises(pkg.PsgldError) as e:
        small.submit(wls[0], N_ITER)
    assert e.value.status == pkg.PSGLD_E_ARG
    small.close()
    srv.close()


def test_served_jobs_track_the_oracle():
    """Jobs served in a mix against the FP64 oracle run of each job: over 40
    iterations (burn-in 12, thinning 2) FP32 and FP64 chains stay close, so
    each job's posterior mean and variance and its held-out RMSE agree
    with the oracle's (rtol 1e-4, as for a context stepped alone)."""
    import oracle
    from parity import oracle_config
    wls = _mix()
    srv = pkg.Server(hbm_budget=8 << 30, max_active=4, iters_per_tick=7)
    ids = [srv.submit(wl, N_ITER, dense=_is_dense(wl), dense_min_cols=1) for wl in wls]
    _drain(srv)
    for jid, wl in zip(ids, wls):
        Wm, Hm, Wv, Hv, rmse = srv.result(jid)
        ch = oracle.Chain(oracle_config(wl), wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
        ch.run(N_ITER)
        rW, rH = ch.posterior_mean()
        qW, qH = ch.posterior_var()
        # the BF16-free dense job runs FP32 MFMA products: same tolerance
        np.testing.assert_allclose(Wm, rW, rtol=1e-4, atol=1e-6)
        np.testing.assert_allclose(Hm, rH, rtol=1e-4, atol=1e-6)
        assert np.all(np.abs(Wv - qW) <= 1e-4 * (rW ** 2 + qW) + 1e-9)
        assert np.all(np.abs(Hv - qH) <= 1e-4 * (rH ** 2 + qH) + 1e-9)
        assert rmse == pytest.approx(ch.heldout_rmse(wl.hval), rel=1e-4)
        srv.release(jid)
    srv.close()


@pytest.mark.parametrize("precision", [pkg.PSGLD_BF16_DENSE, pkg.PSGLD_BF16_DENSE_VALUES])
def test_served_bf16_dense_jobs_match_runs_alone(precision):
    """Dense jobs with BF16 operands, and with BF16-stored values, served
    beside a coordinate job: bitwise the same moments and held-out RMSE as
    the same runs alone."""
    wls = [dense_case(128, 300, 16, 2, 0.5, density=0.9, seed=62),
           dense_case(130, 700, 64, 2, 1.0, density=0.95, seed=63),
           workloads.random_sparse(400, 300, 9000, 8, 4, beta=1.0, prior="exponential", mirror=True,
                                   data_seed=64, chain_seed=65)]
    for wl in wls:
        wl.burn_in, wl.thin = 12, 2
    srv = pkg.Server(hbm_budget=8 << 30, max_active=4, iters_per_tick=7)
    ids = [srv.submit(wl, N_ITER, dense=_is_dense(wl), precision=precision, dense_min_cols=1) for wl in wls]
    _drain(srv)
    for jid, wl in zip(ids, wls):
        assert srv.info(jid)["state"] == pkg.PSGLD_JOB_DONE, srv.error(jid)
        Wm, Hm, _, _, rmse = srv.result(jid)
        s = pkg.PSGLD.from_workload(wl, dense=_is_dense(wl), precision=precision, dense_min_cols=1)
        s.step(N_ITER, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        aWm, aHm = s.posterior_mean()
        assert np.array_equal(Wm, aWm) and np.array_equal(Hm, aHm)
        assert rmse == s.heldout_rmse()
        s.close()
        srv.release(jid)
    srv.close()
