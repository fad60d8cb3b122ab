"""Items cut over many work-groups, at the column skew of the large ratings
workload (Zipf(1.1) columns, K = 100).

With few entries per lane group (entries_per_group = 16), a head column of a
block holds some 100,000 entries and is cut into a few hundred shares, each
a work-group; the share to finish last sums every share's partial gradient
from device memory in slot order.  Stepping the chain for many iterations,
every single step is compared element by element with the FP64 oracle's
step from the same state (stopping at the first iteration that differs), so
a share that read a stale or missing partial fails at once.  The same run
with few large shares must agree within the FP32 tolerance, and repeated
runs are bitwise identical."""
import numpy as np
import pytest

import oracle
import paper_1506_01418_amd as pkg
import workloads
from parity import TOL_FP32, oracle_config, scaled_error

pytestmark = pytest.mark.gpu


def _skewed():
    return workloads.sparse_ratings(I=60_000, J=2_000, nnz=3_000_000, K_true=30, K=100, B=4, zipf_a=1.1,
                                    data_seed=1104, chain_seed=2104, name="skewed_60k")


@pytest.mark.timeout(300)
def test_many_shares_per_item_track_the_oracle_step_by_step():
    wl = _skewed()
    s = pkg.PSGLD.from_workload(wl)
    s.tune(wl.eps_a, wl.eps_t0, wl.eps_gamma, candidates=(16,))
    rp = oracle.partition(wl.I, wl.B)
    per_block_col = np.bincount(rp[wl.row] * wl.J + wl.col, minlength=wl.B * wl.J)
    assert per_block_col.max() > 20 * 32 * 16       # over 20 shares of 32 groups x 16 entries
    ch = oracle.Chain(oracle_config(wl), wl.row, wl.col, wl.val, wl.W0, wl.H0)
    for it in range(24):
        Wg, Hg = s.factors()
        ch.set_state(Wg, Hg, s.iteration())
        bW, bH = ch.run(1, bounds=True)
        s.step(1, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        Wn, Hn = s.factors()
        err = max(float(scaled_error(Wn, ch.W, bW).max()), float(scaled_error(Hn, ch.H, bH).max()))
        assert err <= TOL_FP32, (it, err)
    s.close()


def test_share_count_does_not_change_the_chain_beyond_rounding():
    wl = _skewed()
    runs = []
    for epg in (16, 16, 1024):
        s = pkg.PSGLD.from_workload(wl)
        s.tune(wl.eps_a, wl.eps_t0, wl.eps_gamma, candidates=(epg,))
        s.step(40, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        runs.append(s.factors())
        s.close()
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)                          # bitwise repeatable
    for a, b in zip(runs[0], runs[2]):
        assert np.max(np.abs(a - b)) <= 1e-3 * max(1.0, float(np.max(np.abs(b)))), np.max(np.abs(a - b))
