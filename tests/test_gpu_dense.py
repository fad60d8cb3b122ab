"""GPU-vs-oracle parity of the dense-block path (MFMA), through the C ABI.

psgld_load_dense runs blocks whose training density exceeds the threshold
(and that have at most 128 rows) on the matrix-core kernels; the oracle sees
the same training cells as coordinates.  FP32 operands are held to the FP32
single-step bound, BF16 operands to the BF16 bound."""
import numpy as np
import pytest

import oracle
import paper_1506_01418_amd as pkg
import workloads
import dataclasses

from parity import TOL_BF16, TOL_FP32, bf16_round, oracle_config, step_parity

pytestmark = pytest.mark.gpu


def dense_case(I, J, K, B, beta, density=0.9, seed=0, prior="exponential", mirror=True, block_density=None):
    """A dense-matrix workload; block_density(b, c) overrides the density."""
    rng = np.random.default_rng(seed)
    Wt = rng.gamma(2.0, 0.5, (I, max(2, K // 2)))
    Ht = rng.gamma(1.0, 1.0, (max(2, K // 2), J))
    mu = Wt @ Ht
    V = (mu * rng.gamma(4.0, 0.25, (I, J)) + 0.05).astype(np.float32)
    rp, cp = oracle.partition(I, B), oracle.partition(J, B)
    dens = np.full((I, J), density)
    if block_density is not None:
        dens = np.array([[block_density(rp[i], cp[j]) for j in range(J)] for i in range(I)])
    u = rng.random((I, J))
    mask = (u < dens).astype(np.uint8)
    held = (u >= dens) & (u < dens + 0.05)
    row, col = np.nonzero(mask)
    hrow, hcol = np.nonzero(held)
    val = V[row, col]
    W0, H0 = workloads.init_factors(np.random.default_rng(seed + 1), I, J, K, float(val.mean()), mirror)
    a = workloads.step_scale(row, col, val, I, J, beta, 1.0)
    return workloads.Workload("dense_case", I, J, K, B, beta, 1.0, prior, 1.0, 1.0, mirror, a, 1.0, 0.51,
                              seed + 2, 10, 0, 1, row.astype(np.int32), col.astype(np.int32), val,
                              hrow.astype(np.int32), hcol.astype(np.int32), V[hrow, hcol], W0, H0,
                              dense=V, mask=mask)


@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("steps_before", [0, 5])
def test_dense_poisson_256_parity(bf16, steps_before):
    wl = workloads.dense_poisson()
    prec = pkg.PSGLD_BF16_DENSE if bf16 else pkg.PSGLD_FP32
    err, s = step_parity(wl, steps_before, dense=True, precision=prec)
    s.close()
    assert err <= (TOL_BF16 if bf16 else TOL_FP32), err


@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("case", ["cpois_K64_m65", "gauss_K20_ragged", "gamma_K8_B5", "unequal_heights",
                                  "kl_K48_m128"])
def test_dense_parity_shapes(case, bf16):
    wl = {"cpois_K64_m65": lambda: dense_case(130, 1000, 64, 2, 0.5, seed=1),
          "gauss_K20_ragged": lambda: dense_case(201, 333, 20, 3, 2.0, seed=2, prior="gaussian",
                                                 mirror=False),
          "gamma_K8_B5": lambda: dense_case(150, 170, 8, 5, 0.0, seed=3),
          # pieces of 33, 32 and 32 rows: blocks of one part pad to different heights
          "unequal_heights": lambda: dense_case(97, 400, 16, 3, 1.0, seed=9),
          # the tallest blocks (128 rows: four G_W row tiles per wave, two
          # sub-tiles per work-group) and K = 48 (with FP32 operands one
          # wave in four has no k-tile)
          "kl_K48_m128": lambda: dense_case(256, 600, 48, 2, 1.0, seed=11)}[case]()
    prec = pkg.PSGLD_BF16_DENSE if bf16 else pkg.PSGLD_FP32
    for steps in (0, 4):
        err, s = step_parity(wl, steps, dense=True, precision=prec)
        s.close()
        assert err <= (TOL_BF16 if bf16 else TOL_FP32), (case, steps, err)


def test_mixed_dense_and_sparse_blocks():
    """Diagonal blocks dense, the others below the threshold: each part mixes
    the dense kernels and the coordinate kernel."""
    wl = dense_case(256, 240, 16, 4, 1.0, seed=4, block_density=lambda b, c: 0.8 if b == c else 0.1)
    s = pkg.PSGLD.from_workload(wl, dense=True, dense_min_cols=1)
    for t in range(6):
        err, _ = step_parity(wl, 0, sampler=s)
        assert err <= TOL_FP32, (t, err)
    s.close()


def test_tall_blocks_fall_back_to_coordinates():
    wl = dense_case(300, 90, 12, 2, 1.0, seed=5)      # 150 rows per block > 128
    err, s = step_parity(wl, 3, dense=True)
    s.close()
    assert err <= TOL_FP32


def test_dense_heldout_moments_and_loglik():
    wl = dense_case(160, 400, 16, 4, 1.0, seed=6)
    wl.burn_in, wl.thin = 4, 2
    s = pkg.PSGLD.from_workload(wl, dense=True, dense_min_cols=1)
    s.step(16, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    ch = oracle.Chain(oracle_config(wl), wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
    ch.run(16)
    np.testing.assert_allclose(s.heldout_predictions(), ch.heldout_prediction(), rtol=1e-4)
    mW, mH = s.posterior_mean()
    rW, rH = ch.posterior_mean()
    np.testing.assert_allclose(mW, rW, rtol=1e-4, atol=1e-6)
    np.testing.assert_allclose(mH, rH, rtol=1e-4, atol=1e-6)
    n_p, N = s.part_sizes()
    assert N == len(wl.row) and np.array_equal(n_p, ch.part_sizes())
    Wg, Hg = s.factors()
    ref = oracle.Chain(oracle_config(wl), wl.row, wl.col, wl.val, Wg, Hg)
    assert s.log_likelihood() == pytest.approx(ref.loglik(), rel=1e-10)
    with pytest.raises(pkg.PsgldError):
        t = pkg.PSGLD.from_workload(wl, dense=True, dense_min_cols=1)
        t.load_heldout(wl.row[:2], wl.col[:2])      # training cells
    s.close()


def test_dense_kernels_are_the_ones_running():
    """The precision option only affects dense blocks: if the dense kernels
    run, BF16 and FP32 operands give different bits; for a context whose
    blocks are all below the threshold they give the same bits."""
    wl = dense_case(128, 300, 16, 2, 1.0, seed=8)
    outs = {}
    for thr in (0.3, 0.99):
        for prec in (pkg.PSGLD_FP32, pkg.PSGLD_BF16_DENSE):
            s = pkg.PSGLD.from_workload(wl, dense=True, precision=prec, dense_threshold=thr, dense_min_cols=1)
            s.step(2, wl.eps_a, wl.eps_t0, wl.eps_gamma)
            outs[thr, prec] = s.factors()[0]
            s.close()
    assert not np.array_equal(outs[0.3, pkg.PSGLD_FP32], outs[0.3, pkg.PSGLD_BF16_DENSE])
    assert np.array_equal(outs[0.99, pkg.PSGLD_FP32], outs[0.99, pkg.PSGLD_BF16_DENSE])


def test_dense_runs_are_bitwise_reproducible():
    wl = dense_case(130, 700, 64, 2, 0.5, seed=7)
    out = []
    for _ in range(2):
        s = pkg.PSGLD.from_workload(wl, dense=True, precision=pkg.PSGLD_BF16_DENSE, dense_min_cols=1)
        s.step(4, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        out.append(s.factors())
        s.close()
    assert all(np.array_equal(a, b) for a, b in zip(*out))


def test_bf16_chain_matches_fp32_heldout_rmse():
    """BF16 operands (and BF16-stored values) against FP32 operands on the
    same device: the 1025-row Tweedie spectrogram shape (beta = 0.5, K = 64,
    B = 16) on 4,000 columns, 400 iterations with burn-in 200, every block on
    the dense kernels.  The held-out RMSE of the posterior-mean predictor
    agrees within 1%, and every chain improves on the initial factors' RMSE."""
    wl = workloads.dense_tweedie(J=4000, T=400, burn_in=200, name="dense_tweedie_1025x4k")
    rmse = {}
    for prec in (pkg.PSGLD_FP32, pkg.PSGLD_BF16_DENSE, pkg.PSGLD_BF16_DENSE_VALUES):
        s = pkg.PSGLD.from_workload(wl, dense=True, precision=prec, dense_min_cols=1)
        s.step(wl.T, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        assert s.num_samples() == wl.T - wl.burn_in
        rmse[prec] = s.heldout_rmse()
        s.close()
    mu0 = np.einsum("nk,kn->n", wl.W0[wl.hrow].astype(np.float64), wl.H0[:, wl.hcol].astype(np.float64))
    rmse0 = float(np.sqrt(np.mean((wl.hval - mu0) ** 2)))
    f32 = rmse[pkg.PSGLD_FP32]
    for prec in (pkg.PSGLD_BF16_DENSE, pkg.PSGLD_BF16_DENSE_VALUES):
        assert abs(rmse[prec] - f32) / f32 <= 0.01, (prec, f32, rmse[prec])
    assert all(r < rmse0 for r in rmse.values()), (rmse, rmse0)


def rounded_values(wl):
    """The workload with its training values (dense matrix and entries)
    rounded to BF16; held-out values unchanged."""
    return dataclasses.replace(wl, dense=bf16_round(wl.dense), val=bf16_round(wl.val))


def test_bf16_values_are_rounded_once_to_nearest_even():
    """PSGLD_BF16_DENSE_VALUES stores the dense blocks' training values in
    BF16: a chain given FP32 values steps to the same bits as one given the
    values already rounded to nearest even (by the test's own rounding), and
    as the BF16-operand chain with FP32 storage of those rounded values, which
    reads them exactly; with the unrounded values the BF16-operand chain
    differs, so the rounding is what the storage changes."""
    wl = dense_case(130, 700, 64, 2, 0.5, seed=12)
    wr = rounded_values(wl)
    assert not np.array_equal(wr.val, wl.val)
    out = {}
    for name, w, prec in (("v16", wl, pkg.PSGLD_BF16_DENSE_VALUES), ("v16_rounded", wr, pkg.PSGLD_BF16_DENSE_VALUES),
                          ("v32_rounded", wr, pkg.PSGLD_BF16_DENSE), ("v32", wl, pkg.PSGLD_BF16_DENSE)):
        s = pkg.PSGLD.from_workload(w, dense=True, precision=prec, dense_min_cols=1)
        s.step(5, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        out[name] = s.factors() + (s.log_likelihood(),)
        s.close()
    for name in ("v16_rounded", "v32_rounded"):
        assert all(np.array_equal(a, b) for a, b in zip(out["v16"][:2], out[name][:2])), name
        assert out["v16"][2] == out[name][2], name
    assert not np.array_equal(out["v16"][0], out["v32"][0])


@pytest.mark.parametrize("case", ["cpois_K64_m65", "gauss_K20_ragged"])
def test_bf16_values_parity(case):
    """Single steps with BF16-stored values against the oracle on the same
    rounded values (the chain's data), at the BF16 bound."""
    wl = {"cpois_K64_m65": lambda: dense_case(130, 1000, 64, 2, 0.5, seed=1),
          "gauss_K20_ragged": lambda: dense_case(201, 333, 20, 3, 2.0, seed=2, prior="gaussian",
                                                 mirror=False)}[case]()
    wr = rounded_values(wl)
    for steps in (0, 4):
        err, s = step_parity(wr, steps, dense=True, precision=pkg.PSGLD_BF16_DENSE_VALUES)
        s.close()
        assert err <= TOL_BF16, (case, steps, err)


@pytest.mark.parametrize("bf16", [False, True])
def test_dense_1000_iterations_rmse_parity(bf16):
    """The Poisson NMF chain of 256 x 256 (K = 8, B = 4) for 1000 iterations
    with burn-in 500, every block on the dense kernels: held-out RMSE of the
    posterior-mean predictor within 1% of the oracle's, with FP32 and with
    BF16 operands."""
    wl = workloads.dense_poisson(T=1000, burn_in=500)
    prec = pkg.PSGLD_BF16_DENSE if bf16 else pkg.PSGLD_FP32
    s = pkg.PSGLD.from_workload(wl, dense=True, precision=prec, dense_min_cols=1)
    s.step(wl.T, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    ch = oracle.Chain(oracle_config(wl), wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
    ch.run(wl.T)
    assert s.num_samples() == ch.n_kept == 500
    g, r = s.heldout_rmse(), ch.heldout_rmse(wl.hval)
    s.close()
    assert abs(g - r) <= 0.01 * r, (g, r)
