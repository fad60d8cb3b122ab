"""The paper's synthetic shared-memory experiments (Section 4.2.1) as
synthetic stand-ins: Poisson NMF of a fully observed 512 x 512 matrix
(K = 32, B = I / 32 = 16) and the compound Poisson (beta = 0.5, phi = 1)
1024 x 1024 case (K = 32, B = 32), each 10,000 iterations.

Single steps are compared element by element with the FP64 oracle, and the
mixing indicator the paper plots -- the training log-likelihood of the
chain's state every 100 iterations -- is compared with the oracle's stored
trace of the same whole run: close while the two chains still agree (the
first few hundred iterations), and at the same level over the second half,
where FP32 and FP64 chains have long become different samples of the same
posterior."""
import json
import os

import numpy as np
import pytest

import paper_1506_01418_amd as pkg
import workloads
from parity import TOL_FP32, step_parity

pytestmark = pytest.mark.gpu

NAMES = ["paper_poisson_512", "paper_cpoisson_1024"]


@pytest.mark.parametrize("name", NAMES)
def test_paper_shape_step_parity(name):
    wl = workloads.by_name(name)
    err0, s = step_parity(wl, 0)
    err1, _ = step_parity(wl, 36, sampler=s)
    s.close()
    assert err0 <= TOL_FP32 and err1 <= TOL_FP32, (err0, err1)


@pytest.mark.parametrize("name", NAMES)
def test_paper_shape_mixing_trace_matches_oracle(name):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ll_trace.json")
    with open(path) as f:
        ref = json.load(f)[name]
    wl = workloads.by_name(name)
    assert ref["T"] == wl.T and ref["nnz"] == wl.nnz
    s = pkg.PSGLD.from_workload(wl)
    pts = [[0, s.log_likelihood()]]
    while s.iteration() < wl.T:
        s.step(ref["every"], wl.eps_a, wl.eps_t0, wl.eps_gamma)
        pts.append([s.iteration(), s.log_likelihood()])
    s.close()
    g = np.array(pts, dtype=np.float64)
    r = np.array(ref["points"], dtype=np.float64)
    assert np.array_equal(g[:, 0], r[:, 0])
    early = slice(0, 4)                       # t = 0 .. 300
    np.testing.assert_allclose(g[early, 1], r[early, 1], rtol=1e-4)
    late = g[:, 0] > wl.T // 2
    gm, rm = g[late, 1].mean(), r[late, 1].mean()
    assert abs(gm - rm) <= 0.01 * abs(rm), (gm, rm)
    # the chain has mixed: the late level is far above the starting point
    assert gm > g[0, 1] and rm > r[0, 1]
