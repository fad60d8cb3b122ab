"""Random part order (Condition 2): the part of every iteration is drawn
with probability |part| / N from the PART Philox stream, on the host in the
library and independently in the oracle.  Single steps and a 200-iteration
chain match the oracle; every launch mode gives the same bits."""
import numpy as np
import pytest

import oracle
import paper_1506_01418_amd as pkg
import workloads
from parity import TOL_FP32, oracle_config, step_parity

pytestmark = pytest.mark.gpu


def _zipf():
    return workloads.random_sparse(2000, 700, 60_000, 24, 6, beta=2.0, phi=0.5, zipf_a=1.0,
                                   data_seed=91, chain_seed=92)


@pytest.mark.parametrize("steps_before", [0, 7])
def test_random_order_step_parity(steps_before):
    wl = _zipf()
    err, s = step_parity(wl, steps_before, part_order="random")
    s.close()
    assert err <= TOL_FP32, err


@pytest.mark.parametrize("bf16", [False, True])
def test_random_order_dense_and_mixed_blocks(bf16):
    """Random order over parts that mix dense blocks (MFMA kernels) and
    coordinate blocks: the drawn part decides which blocks and which scale
    each iteration uses on both paths."""
    from test_gpu_dense import dense_case
    # row pieces 0 and 2 dense, 1 and 3 sparse: every part has both kinds
    wl = dense_case(150, 700, 32, 4, 0.5, density=0.85, seed=95,
                    block_density=lambda b, c: 0.85 if b % 2 == 0 else 0.1)
    prec = pkg.PSGLD_BF16_DENSE if bf16 else pkg.PSGLD_FP32
    from parity import TOL_BF16
    for steps in (0, 6):
        err, s = step_parity(wl, steps, dense=True, precision=prec, part_order="random")
        s.close()
        assert err <= (TOL_BF16 if bf16 else TOL_FP32), (steps, err)


def test_random_order_launch_modes_agree():
    wl = _zipf()
    kw = dict(burn_in=5, thin=2, part_order="random")
    eager = pkg.PSGLD.from_workload(wl, graph_iters=-1, **kw)
    auto = pkg.PSGLD.from_workload(wl, **kw)                       # graphs are not used in random order
    pers = pkg.PSGLD.from_workload(wl, persistent=1, **kw)
    other = workloads.random_sparse(500, 400, 9000, 8, 3, beta=1.0, prior="exponential", mirror=True,
                                    data_seed=93, chain_seed=94)
    first = pkg.PSGLD.from_workload(wl, **kw)
    second = pkg.PSGLD.from_workload(other, stream=first.stream(), **kw)
    alone2 = pkg.PSGLD.from_workload(other, **kw)
    for n in (3, 40, 1, 20):
        for s in (eager, auto, pers):
            s.step(n, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        alone2.step(n, other.eps_a, other.eps_t0, other.eps_gamma)
        pkg.PSGLD.step_batch([first, second], [n, n], [(wl.eps_a, wl.eps_t0, wl.eps_gamma),
                                                       (other.eps_a, other.eps_t0, other.eps_gamma)])
    ref = (*eager.factors(), *eager.posterior_mean(), eager.heldout_predictions())
    for s in (auto, pers, first):
        got = (*s.factors(), *s.posterior_mean(), s.heldout_predictions())
        for x, y in zip(ref, got):
            assert np.array_equal(x, y, equal_nan=True)
    for x, y in zip((*alone2.factors(), alone2.heldout_predictions()),
                    (*second.factors(), second.heldout_predictions())):
        assert np.array_equal(x, y, equal_nan=True)
    for s in (second, first, alone2, pers, auto, eager):
        s.close()


def test_random_order_200_iterations_rmse_parity():
    """The Poisson NMF chain of 256 x 256, K = 8, B = 4 in random part order:
    held-out RMSE of the posterior-mean predictor within 1% of the oracle's."""
    wl = workloads.dense_poisson()
    s = pkg.PSGLD.from_workload(wl, part_order="random")
    s.step(wl.T, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    ch = oracle.Chain(oracle_config(wl, part_order="random"), wl.row, wl.col, wl.val, wl.W0, wl.H0,
                      wl.hrow, wl.hcol)
    ch.run(wl.T)
    g, r = s.heldout_rmse(), ch.heldout_rmse(wl.hval)
    s.close()
    assert abs(g - r) <= 0.01 * r, (g, r)
