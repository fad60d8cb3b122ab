"""Captured iteration graphs: a run of graph_iters iterations is captured
once per (first part, ping-pong buffer) and replayed; each replay reads its
iteration from the device clock and its step sizes from the device table.
Replays must give the same bits as launching the iterations one at a time,
across calls of any length, schedule changes, checkpoints and both the
coordinate and the dense-block kernels."""
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


def _zipf_case():
    return workloads.random_sparse(1200, 700, 40_000, 24, 5, beta=2.0, phi=0.5, prior="gaussian",
                                   zipf_a=1.0, data_seed=11, chain_seed=12)


@pytest.mark.parametrize("graph_iters", [0, 7, 10])
def test_graph_replays_match_single_launches(graph_iters):
    wl = _zipf_case()
    eager = pkg.PSGLD.from_workload(wl, burn_in=9, thin=3, graph_iters=-1)
    graph = pkg.PSGLD.from_workload(wl, burn_in=9, thin=3, graph_iters=graph_iters)
    # call lengths below, at and above the graph length, from shifting phases
    for n in (3, 40, 1, 21, 7, 35):
        eager.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        graph.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    _assert_same(eager, graph)
    eager.close()
    graph.close()


def test_graph_after_schedule_change_and_checkpoint():
    wl = _zipf_case()
    eager = pkg.PSGLD.from_workload(wl, burn_in=4, graph_iters=-1)
    graph = pkg.PSGLD.from_workload(wl, burn_in=4, graph_iters=10)
    for s in (eager, graph):
        s.step(30, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        s.step(30, 0.5 * wl.eps_a, 3.0, 0.75)       # new schedule: table refilled
    _assert_same(eager, graph)
    state = eager.get_state()
    resumed = pkg.PSGLD.from_workload(wl, burn_in=4, graph_iters=10)
    resumed.step(10, wl.eps_a, wl.eps_t0, wl.eps_gamma)  # clock moves elsewhere first
    resumed.set_state(state)
    for s in (eager, resumed):
        s.step(25, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    _assert_same(eager, resumed)
    for s in (eager, graph, resumed):
        s.close()


@pytest.mark.parametrize("bf16", [False, True])
def test_graph_dense_blocks_match_single_launches(bf16):
    wl = dense_case(150, 700, 32, 4, 0.5, density=0.85, seed=21,
                    block_density=lambda b, c: 0.85 if (b + c) % 2 == 0 else 0.1)
    prec = pkg.PSGLD_BF16_DENSE if bf16 else pkg.PSGLD_FP32
    eager = pkg.PSGLD.from_workload(wl, dense=True, precision=prec, burn_in=6, graph_iters=-1,
                                  dense_min_cols=1)
    graph = pkg.PSGLD.from_workload(wl, dense=True, precision=prec, burn_in=6, graph_iters=8,
                                  dense_min_cols=1)
    for n in (5, 17, 8, 2):
        eager.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        graph.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    _assert_same(eager, graph)
    eager.close()
    graph.close()


def test_graph_state_keeps_single_step_parity():
    """After graph replays the next iteration still matches the oracle."""
    wl = _zipf_case()
    s = pkg.PSGLD.from_workload(wl, graph_iters=10)
    err, s = step_parity(wl, 20, sampler=s)
    assert err <= TOL_FP32, err
    s.close()
