"""GPU-vs-oracle parity of the HIP sampler, through the C ABI.

Single steps are compared element by element at t = 0 and at a mid-run t
(the GPU's FP32 state handed to the oracle), against the tolerance of
parity.TOL_FP32.  Cases span every kernel variant (lanes per group 1..64,
each likelihood branch), ragged shapes, Zipf-skewed items long enough to be
split over several groups, empty parts and rows, custom partitions and the
test flags."""
import numpy as np
import pytest

import oracle
import paper_1506_01418_amd as pkg
import workloads
from parity import TOL_FP32, oracle_config, philox_kat, scaled_error, step_parity

pytestmark = pytest.mark.gpu


# ------------------------------------------------------------------ noise stream
def test_philox_blocks_bit_exact():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, (2000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, (2000, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    key[0] = 0
    got = pkg.psgld_philox_blocks(ctr, key)
    for c, k, g in zip(ctr, key, got):
        assert np.array_equal(oracle.philox4x32_10(c, k), g)


def test_philox_blocks_known_answer_vectors():
    inp, expect = philox_kat()
    got = pkg.psgld_philox_blocks(inp[:, :4], inp[:, 4:])
    assert np.array_equal(got, expect), (got, expect)


def test_normals_match_oracle():
    rng = np.random.default_rng(1)
    n, K = 3000, 13
    t = rng.integers(0, 5000, n)
    st = rng.integers(0, 2, n).astype(np.uint32)
    idx = rng.integers(0, 500_000, n)
    z, r = pkg.psgld_normals(1234567, t, st, idx, K)
    for m in range(n):
        zr, rr = oracle.normals(1234567, int(t[m]), int(st[m]), int(idx[m]), K)
        np.testing.assert_allclose(r[m], rr, rtol=2e-6)
        assert np.all(np.abs(z[m] - zr) <= 2e-6 * rr), m


# ------------------------------------------------------------------ single steps
CASES = {
    # name: workload factory
    "gauss_K50_zipf": lambda: workloads.random_sparse(
        3000, 800, 150_000, 50, 4, beta=2.0, phi=0.5, prior="gaussian", zipf_a=1.0,
        data_seed=1, chain_seed=2),
    "poisson_K8_dense256": lambda: workloads.dense_poisson(),
    "cpois_K64_B16": lambda: workloads.random_sparse(
        700, 900, 120_000, 64, 16, beta=0.5, prior="exponential", mirror=True, zipf_a=0.8,
        data_seed=3, chain_seed=4),
    "gamma_K5_B3": lambda: workloads.random_sparse(
        301, 199, 9000, 5, 3, beta=0.0, prior="exponential", mirror=True, data_seed=5,
        chain_seed=6),
    "K1_B1": lambda: workloads.random_sparse(50, 40, 600, 1, 1, beta=2.0, data_seed=7,
                                             chain_seed=8),
    "K100_B8": lambda: workloads.random_sparse(1500, 1100, 80_000, 100, 8, beta=2.0, phi=0.4,
                                               zipf_a=1.1, data_seed=9, chain_seed=10),
    "K256_B2": lambda: workloads.random_sparse(120, 90, 3000, 256, 2, beta=1.0,
                                               prior="exponential", mirror=True, data_seed=11,
                                               chain_seed=12),
    "K3_ragged_B7": lambda: workloads.random_sparse(103, 59, 1500, 3, 7, beta=2.0,
                                                    data_seed=13, chain_seed=14),
    "K30_gauss_mirror": lambda: workloads.random_sparse(400, 300, 20_000, 30, 5, beta=2.0,
                                                        prior="gaussian", mirror=True,
                                                        data_seed=15, chain_seed=16),
    # four quads per lane over 8 lanes (32 quads) on rows of 96 floats: the
    # last lanes' partner reads run past the row and are masked
    "K68_B4": lambda: workloads.random_sparse(600, 500, 20_000, 68, 4, beta=2.0, phi=0.5, zipf_a=1.0,
                                              data_seed=19, chain_seed=20),
    # general beta (no closed-form branch) with 4 lanes of one quad each
    "K12_beta07_B5": lambda: workloads.random_sparse(500, 420, 25_000, 12, 5, beta=0.7,
                                                     prior="exponential", mirror=True, zipf_a=1.0,
                                                     data_seed=17, chain_seed=18),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("steps_before", [0, 7])
def test_single_step_parity(name, steps_before):
    wl = CASES[name]()
    err, s = step_parity(wl, steps_before)
    s.close()
    assert err <= TOL_FP32, (name, steps_before, err)


@pytest.mark.parametrize("flags", [pkg.PSGLD_TEST_NOISE_OFF, pkg.PSGLD_TEST_FREEZE_W,
                                   pkg.PSGLD_TEST_FREEZE_H,
                                   pkg.PSGLD_TEST_NOISE_OFF | pkg.PSGLD_TEST_FREEZE_H])
def test_single_step_parity_test_flags(flags):
    wl = CASES["gauss_K50_zipf"]()
    err, s = step_parity(wl, 3, flags=flags)
    s.close()
    assert err <= TOL_FP32


def test_empty_parts_and_rows():
    """Entries only on the diagonal blocks: parts 1..B-1 are empty (scale 0,
    prior and noise only); many rows and columns have no entry at all."""
    I, J, K, B = 200, 160, 12, 4
    rng = np.random.default_rng(3)
    rp, cp = oracle.partition(I, B), oracle.partition(J, B)
    keys = rng.choice(I * J, 6000, replace=False)
    r, c = keys // J, keys % J
    keep = rp[r] == cp[c]
    wl = workloads.random_sparse(I, J, 10, K, B, data_seed=4, chain_seed=5)
    wl.row, wl.col = r[keep].astype(np.int32), c[keep].astype(np.int32)
    wl.val = rng.gamma(2.0, 1.0, keep.sum()).astype(np.float32)
    wl.hrow, wl.hcol, wl.hval = wl.hrow[:0], wl.hcol[:0], wl.hval[:0]
    s = pkg.PSGLD.from_workload(wl)
    n_p, N = s.part_sizes()
    assert N == keep.sum() and n_p[0] == N and np.all(n_p[1:] == 0)
    for t in range(B + 1):
        err, _ = step_parity(wl, 0, sampler=s)
        assert err <= TOL_FP32, (t, err)
    s.close()


def test_no_training_entries():
    wl = workloads.random_sparse(64, 48, 10, 8, 4, data_seed=6, chain_seed=7)
    wl.row, wl.col, wl.val = wl.row[:0], wl.col[:0], wl.val[:0]
    wl.hrow, wl.hcol, wl.hval = wl.hrow[:0], wl.hcol[:0], wl.hval[:0]
    err, s = step_parity(wl, 2)
    s.close()
    assert err <= TOL_FP32


def test_custom_partitions():
    """Data-dependent partitions (Section 3: blocks need not come from a
    regular grid): random piece maps."""
    wl = workloads.random_sparse(500, 350, 20_000, 16, 5, beta=2.0, data_seed=8, chain_seed=9)
    rng = np.random.default_rng(2)
    rp = rng.permutation(np.arange(wl.I) % wl.B).astype(np.int32)
    cp = rng.permutation(np.arange(wl.J) % wl.B).astype(np.int32)
    err, s = step_parity(wl, 4, row_piece=rp, col_piece=cp)
    s.close()
    assert err <= TOL_FP32


# ------------------------------------------------------------------ chains
def test_moments_and_heldout_track_oracle():
    """30 iterations with burn-in and thinning run independently on both
    sides from the same start; FP32 and FP64 chains stay close over so few
    steps, so posterior moments and held-out predictions agree closely."""
    wl = workloads.random_sparse(600, 500, 30_000, 10, 5, beta=1.0, prior="exponential",
                                 mirror=True, data_seed=20, chain_seed=21)
    wl.burn_in, wl.thin = 10, 3
    s = pkg.PSGLD.from_workload(wl)
    s.step(30, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    ch = oracle.Chain(oracle_config(wl), wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
    ch.run(30)
    assert s.num_samples() == ch.n_kept == 7
    mW, mH = s.posterior_mean()
    rW, rH = ch.posterior_mean()
    np.testing.assert_allclose(mW, rW, rtol=1e-4, atol=1e-6)
    np.testing.assert_allclose(mH, rH, rtol=1e-4, atol=1e-6)
    vW, vH = s.posterior_var()
    qW, qH = ch.posterior_var()
    assert np.all(np.abs(vW - qW) <= 1e-4 * (rW ** 2 + qW) + 1e-9)
    assert np.all(np.abs(vH - qH) <= 1e-4 * (rH ** 2 + qH) + 1e-9)
    pred = s.heldout_predictions()
    np.testing.assert_allclose(pred, ch.heldout_prediction(), rtol=1e-4)
    assert s.heldout_rmse() == pytest.approx(ch.heldout_rmse(wl.hval), rel=1e-4)
    s.close()


def test_dense_poisson_200_iterations_rmse_parity():
    """The plain dense Poisson NMF chain (I = J = 256, K = 8, B = 4, 200
    iterations, burn-in 100): held-out RMSE of the posterior-mean predictor
    within 1% of the oracle's."""
    wl = workloads.dense_poisson()
    s = pkg.PSGLD.from_workload(wl)
    s.step(wl.T, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    ch = oracle.Chain(oracle_config(wl), wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
    ch.run(wl.T)
    g, r = s.heldout_rmse(), ch.heldout_rmse(wl.hval)
    s.close()
    assert abs(g - r) / r <= 0.01, (g, r)


@pytest.mark.parametrize("case", [
    dict(I=1500, J=800, nnz=100_000, K=20, B=8, beta=2.0, zipf_a=1.0),
    dict(I=1200, J=900, nnz=80_000, K=16, B=6, beta=1.0, prior="exponential", mirror=True, zipf_a=1.0),
], ids=["gauss_K20_B8", "kl_K16_B6"])
def test_1000_iterations_rmse_parity(case):
    """1000 iterations with burn-in 500 and thinning 5 (Zipf-skewed columns):
    held-out RMSE of the posterior-mean predictor within 1% of the oracle's,
    and below the RMSE of the initial factors."""
    a = dict(case)
    I, J, nnz, K, B = (a.pop(k) for k in ("I", "J", "nnz", "K", "B"))
    wl = workloads.random_sparse(I, J, nnz, K, B, data_seed=31, chain_seed=32, T=1000, burn_in=500, thin=5, **a)
    s = pkg.PSGLD.from_workload(wl)
    s.step(wl.T, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    ch = oracle.Chain(oracle_config(wl), wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
    ch.run(wl.T)
    assert s.num_samples() == ch.n_kept == 100
    g, r = s.heldout_rmse(), ch.heldout_rmse(wl.hval)
    s.close()
    mu0 = np.einsum("nk,kn->n", wl.W0[wl.hrow].astype(np.float64), wl.H0[:, wl.hcol].astype(np.float64))
    r0 = float(np.sqrt(np.mean((wl.hval - mu0) ** 2)))
    assert abs(g - r) <= 0.01 * r, (g, r)
    assert r < r0 and g < r0, (g, r, r0)


def test_log_likelihood_matches_oracle():
    wl = CASES["cpois_K64_B16"]()
    s = pkg.PSGLD.from_workload(wl)
    s.step(3, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    Wg, Hg = s.factors()
    ch = oracle.Chain(oracle_config(wl), wl.row, wl.col, wl.val, Wg, Hg)
    assert s.log_likelihood() == pytest.approx(ch.loglik(), rel=1e-10)
    s.close()


def test_runs_are_bitwise_reproducible():
    wl = CASES["gauss_K50_zipf"]()
    out = []
    for _ in range(2):
        s = pkg.PSGLD.from_workload(wl, burn_in=2)
        s.step(6, wl.eps_a, wl.eps_t0, wl.eps_gamma)
        out.append((*s.factors(), s.heldout_predictions(), *s.posterior_mean()))
        s.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b, equal_nan=True)


def test_checkpoint_resume_is_bit_identical():
    wl = CASES["cpois_K64_B16"]()
    a = pkg.PSGLD.from_workload(wl, burn_in=3)
    a.step(10, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    b = pkg.PSGLD.from_workload(wl, burn_in=3)
    b.step(4, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    state = b.get_state()
    b.close()
    c = pkg.PSGLD.from_workload(wl, burn_in=3)
    c.set_state(state)
    assert c.iteration() == 4
    c.step(6, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    for x, y in zip((*a.factors(), *a.posterior_mean(), a.heldout_predictions()),
                    (*c.factors(), *c.posterior_mean(), c.heldout_predictions())):
        assert np.array_equal(x, y, equal_nan=True)
    a.close()
    c.close()


def test_tune_keeps_chain_and_is_reproducible():
    """Tuning times candidate schedules on copies of the state: the chain is
    unchanged, and a context given the chosen value directly steps to the
    same bits.  Every candidate schedule stays within the parity bound."""
    wl = CASES["gauss_K50_zipf"]()
    a = pkg.PSGLD.from_workload(wl)
    a.set_schedule(64)
    a.step(3, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    before = a.factors()
    chosen = a.tune(wl.eps_a, wl.eps_t0, wl.eps_gamma, candidates=(8, 64), iters=4)
    assert chosen in (8, 64)
    epg, qpl, lpg = a.schedule_info()
    assert epg == chosen and qpl in (2, 4) and lpg == {2: 8, 4: 4}[qpl]   # K = 50: 13 quads
    after = a.factors()
    assert all(np.array_equal(x, y) for x, y in zip(before, after)) and a.iteration() == 3
    a.step(5, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    b = pkg.PSGLD.from_workload(wl)   # loads with the choice remembered for this shape
    assert b.schedule_info() == (epg, qpl, lpg)
    b.set_schedule(64)
    b.step(3, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    b.set_schedule(epg, qpl)
    b.step(5, wl.eps_a, wl.eps_t0, wl.eps_gamma)
    assert all(np.array_equal(x, y) for x, y in zip(a.factors(), b.factors()))
    a.close()
    b.close()
    for L, q in ((1, 2), (8, 4), (200, 2), (200, 4)):
        s = pkg.PSGLD.from_workload(wl)
        s.set_schedule(L, q)
        err, _ = step_parity(wl, 2, sampler=s)
        s.close()
        assert err <= TOL_FP32, (L, q, err)


def test_nonfinite_is_reported():
    wl = CASES["K3_ragged_B7"]()
    s = pkg.PSGLD.from_workload(wl)
    s.step(3, 1e30, 1.0, 0.0)
    with pytest.raises(pkg.PsgldError) as e:
        s.sync()
    assert e.value.status == pkg.PSGLD_E_NUMERIC
    s.close()


def test_state_errors():
    wl = CASES["K3_ragged_B7"]()
    s = pkg.PSGLD(wl.I, wl.J, wl.K, wl.B)
    s.load_coo(wl.row, wl.col, wl.val)
    with pytest.raises(pkg.PsgldError) as e:
        s.step(1, 1e-3)                       # factors not set
    assert e.value.status == pkg.PSGLD_E_STATE
    with pytest.raises(pkg.PsgldError) as e:
        s.load_coo(wl.row, wl.col, wl.val)    # second load
    assert e.value.status == pkg.PSGLD_E_STATE
    with pytest.raises(pkg.PsgldError) as e:
        s.load_heldout(wl.row[:3], wl.col[:3])   # overlaps training
    assert e.value.status == pkg.PSGLD_E_STATE
    with pytest.raises(pkg.PsgldError) as e:
        s.posterior_mean()                    # no samples
    assert e.value.status == pkg.PSGLD_E_STATE
    s.close()
    d = pkg.PSGLD(4, 4, 2, 2)
    with pytest.raises(pkg.PsgldError, match="duplicate"):
        d.load_coo([0, 0], [1, 1], [1.0, 2.0])
    d.close()


@pytest.mark.parametrize("K,qpl", [(20, 1), (20, 2), (50, 2), (50, 4), (100, 2), (100, 4), (200, 2), (200, 4)])
def test_every_kernel_variant_step_parity(K, qpl):
    """Each (quads per lane, lanes per group) kernel the tuner may choose for
    a rank steps within the parity bound, before and after burn-in."""
    wl = workloads.random_sparse(900, 700, 40_000, K, 4, beta=2.0, phi=0.5, zipf_a=1.0,
                                 data_seed=40 + K, chain_seed=41 + K, burn_in=3, thin=2)
    s = pkg.PSGLD.from_workload(wl)
    s.set_schedule(32, qpl)
    assert s.schedule_info()[1] == qpl
    err0, _ = step_parity(wl, 0, sampler=s)
    err1, _ = step_parity(wl, 4, sampler=s)
    s.close()
    assert err0 <= TOL_FP32 and err1 <= TOL_FP32, (K, qpl, err0, err1)
