"""The library driven from plain C (tests/c_abi_driver.c): no Python and no
PyTorch in the stepping process.  Its first step is checked against the FP64
oracle, and five steps against the Python binding's, bit for bit (the
binding only marshals arguments)."""
import dataclasses

import numpy as np
import pytest

import oracle
import paper_1506_01418_amd as pkg
import workloads
from c_driver import build_driver, run_driver, write_problem
from parity import TOL_FP32, oracle_config, scaled_error

pytestmark = pytest.mark.gpu


def test_c_program_steps_like_the_oracle_and_the_binding(tmp_path):
    wl = workloads.random_sparse(700, 520, 30_000, 24, 4, beta=1.0, prior="exponential", mirror=True,
                                 zipf_a=1.0, data_seed=41, chain_seed=42)
    wl = dataclasses.replace(wl, burn_in=0, thin=1)
    exe = build_driver(tmp_path)
    write_problem(tmp_path, wl)

    W1, H1, _, _ = run_driver(exe, tmp_path, 1, wl)
    ch = oracle.Chain(oracle_config(wl), wl.row, wl.col, wl.val, wl.W0, wl.H0)
    bW, bH = ch.run(1, bounds=True)
    err = max(float(scaled_error(W1, ch.W, bW).max()), float(scaled_error(H1, ch.H, bH).max()))
    assert err <= TOL_FP32, err

    W5, H5, mW5, mH5 = run_driver(exe, tmp_path, 5, wl)
    s = pkg.PSGLD.from_workload(wl)
    s.step(5, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    Wp, Hp = s.factors()
    mWp, mHp = s.posterior_mean()
    s.close()
    assert np.array_equal(W5, Wp) and np.array_equal(H5, Hp)
    assert np.array_equal(mW5, mWp) and np.array_equal(mH5, mHp)
