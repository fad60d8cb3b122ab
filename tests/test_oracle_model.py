"""Pins of the FP64 oracle against mathematics that does not come from it.

Each test names the passage of the paper it checks.  The numpy code in this
file is written independently of the C oracle (it never calls the oracle's
gradient to check the oracle's gradient).
"""
import numpy as np
import pytest

import oracle
import workloads

BETAS = [0.0, 0.5, 1.0, 2.0]


# ------------------------------------------------------- independent numpy model
def dbeta_np(v, mu, beta):
    """beta-divergence of Section 4 with its KL (beta=1) and IS (beta=0) limits."""
    v = np.asarray(v, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    if beta == 1.0:
        return np.where(v > 0, v * np.log(np.where(v > 0, v, 1.0) / mu), 0.0) - v + mu
    if beta == 0.0:
        return v / mu - np.log(v / mu) - 1.0
    return v ** beta / (beta * (beta - 1)) - v * mu ** (beta - 1) / (beta - 1) + mu ** beta / beta


def log_prior_np(W, H, cfg):
    if cfg.prior == "exponential":   # rate lambda on |x|
        return (np.sum(np.log(cfg.lambda_w) - cfg.lambda_w * np.abs(W)) +
                np.sum(np.log(cfg.lambda_h) - cfg.lambda_h * np.abs(H)))
    return -0.5 * cfg.lambda_w * np.sum(W * W) - 0.5 * cfg.lambda_h * np.sum(H * H)


def part_members(row, col, rp, cp, B, p):
    """Definition 2 with the cyclic family: block (b, (b + p) mod B)."""
    return (rp[row] + p) % B == cp[col]


def log_joint_part_np(W, H, wl_row, wl_col, wl_val, rp, cp, cfg, p):
    """L^_p(theta) = log p(theta) + N/|Pi_p| sum_{Pi_p} log p(v|theta)
    (Section 3.1), the Tweedie normaliser dropped."""
    inp = part_members(wl_row, wl_col, rp, cp, cfg.B, p)
    N, n_p = len(wl_row), int(inp.sum())
    s = N / n_p if n_p else 0.0
    Wm = np.abs(W) if cfg.mirror else W
    Hm = np.abs(H) if cfg.mirror else H
    r, c, v = wl_row[inp], wl_col[inp], wl_val[inp].astype(np.float64)
    mu = np.einsum("nk,kn->n", Wm[r], Hm[:, c])
    if cfg.beta < 2:
        mu = np.maximum(mu, cfg.mu_floor)
    return log_prior_np(W, H, cfg) + s * (-np.sum(dbeta_np(v, mu, cfg.beta)) / cfg.phi)


def small_problem(beta, prior, mirror, seed=0, I=7, J=6, K=3, B=2, nnz=26):
    wl = workloads.random_sparse(I, J, nnz, K, B, beta=beta, phi=0.7, prior=prior,
                                 mirror=mirror, data_seed=seed, chain_seed=seed + 50)
    cfg = oracle.Config(I=I, J=J, K=K, B=B, beta=beta, phi=0.7, prior=prior, lambda_w=1.3,
                        lambda_h=0.8, mirror=mirror, eps_a=1e-3, seed=11)
    ch = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
    return wl, cfg, ch


# ------------------------------------------------------------------- P1
@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("prior,mirror", [("exponential", True), ("gaussian", False),
                                          ("gaussian", True)])
def test_drift_matches_finite_differences(beta, prior, mirror):
    """Eq. (8)-(9): the drift is the gradient of the part-estimated log joint."""
    wl, cfg, ch = small_problem(beta, prior, mirror, seed=int(beta * 10) + 3)
    rp, cp = ch.row_piece, ch.col_piece
    W, H = ch.W.copy(), ch.H.copy()
    for p in range(cfg.B):
        dW, dH = ch.drift(p)
        for X, D, is_w in [(W, dW, True), (H, dH, False)]:
            for idx in np.ndindex(X.shape):
                h = 1e-6 * max(1.0, abs(X[idx]))
                Xp, Xm = X.copy(), X.copy()
                Xp[idx] += h
                Xm[idx] -= h
                args = (Xp, H) if is_w else (W, Xp)
                fp = log_joint_part_np(*args, wl.row, wl.col, wl.val, rp, cp, cfg, p)
                args = (Xm, H) if is_w else (W, Xm)
                fm = log_joint_part_np(*args, wl.row, wl.col, wl.val, rp, cp, cfg, p)
                fd = (fp - fm) / (2 * h)
                assert abs(fd - D[idx]) <= 1e-6 * max(1.0, abs(D[idx])), (p, is_w, idx, fd, D[idx])


# ------------------------------------------------------------------- P2
@pytest.mark.parametrize("n,B", [(10, 3), (256, 4), (70_000, 32), (7, 7), (5, 1)])
def test_partition_is_array_split(n, B):
    """Section 3: P_B(S) holds B non-empty disjoint contiguous pieces."""
    pieces = oracle.partition(n, B)
    ref = np.concatenate([np.full(len(a), b) for b, a in enumerate(np.array_split(np.arange(n), B))])
    assert np.array_equal(pieces, ref)
    assert np.all(np.bincount(pieces, minlength=B) > 0)


@pytest.mark.parametrize("B", [1, 2, 3, 5, 8])
def test_parts_are_disjoint_and_cover_every_block(B):
    """Definition 2 and Condition 2: each part's blocks share no row or column
    piece, and the B parts cover all B^2 blocks exactly once."""
    seen = np.zeros((B, B), dtype=int)
    for p in range(B):
        cols = [(b + p) % B for b in range(B)]
        assert sorted(cols) == list(range(B))
        for b, c in enumerate(cols):
            seen[b, c] += 1
    assert np.all(seen == 1)


def test_part_membership_by_behaviour_figure1():
    """Figure 1 (B = 3): the first part is the three diagonal blocks.  With
    the noise off and H frozen, a step at t = p may depend only on the
    entries inside part p; perturbing any other entry leaves W unchanged."""
    I, J, K, B = 9, 9, 2, 3
    rows, cols = np.meshgrid(np.arange(I), np.arange(J), indexing="ij")
    row, col = rows.ravel().astype(np.int32), cols.ravel().astype(np.int32)
    rng = np.random.default_rng(1)
    val = rng.gamma(2.0, 1.0, I * J)
    W0 = rng.gamma(2.0, 0.5, (I, K))
    H0 = rng.gamma(2.0, 0.5, (K, J))
    cfg = oracle.Config(I=I, J=J, K=K, B=B, beta=2.0, phi=1.0, prior="gaussian",
                        eps_a=1e-2, eps_gamma=0.0, flags=oracle.FLAG_NOISE_OFF | oracle.FLAG_FREEZE_H)
    for p in range(B):
        base = oracle.Chain(cfg, row, col, val, W0, H0)
        base.t = p
        base.run(1)
        for e in range(I * J):
            v2 = val.copy()
            v2[e] += 1.0
            ch = oracle.Chain(cfg, row, col, v2, W0, H0)
            ch.t = p
            ch.run(1)
            inside = (row[e] // 3 + p) % 3 == col[e] // 3
            if p == 0:
                assert inside == (row[e] // 3 == col[e] // 3)   # diagonal blocks
            assert (not np.array_equal(ch.W, base.W)) == inside, (p, e)
        assert base.part_sizes()[p] == 27


# ------------------------------------------------------------------- P4
@pytest.mark.parametrize("beta", [1.0, 2.0])
def test_part_estimates_are_unbiased(beta):
    """Condition 2 / proof sketch of Theorem 1: with p(Pi) = |Pi|/N the part
    gradients average to the full-data gradient."""
    wl, cfg, ch = small_problem(beta, "gaussian", False, seed=5, I=12, J=10, B=3, nnz=70)
    n_p = ch.part_sizes()
    N = n_p.sum()
    assert N == len(wl.row)
    prior_W = -cfg.lambda_w * ch.W
    prior_H = -cfg.lambda_h * ch.H
    avg_W = np.zeros_like(ch.W)
    avg_H = np.zeros_like(ch.H)
    for p in range(cfg.B):
        dW, dH = ch.drift(p)
        avg_W += n_p[p] / N * (dW - prior_W)
        avg_H += n_p[p] / N * (dH - prior_H)
    # full-data likelihood gradient, independently by central differences
    def full_ll(W, H):
        mu = np.einsum("nk,kn->n", W[wl.row], H[:, wl.col])
        if beta < 2:
            mu = np.maximum(mu, cfg.mu_floor)
        return -np.sum(dbeta_np(wl.val, mu, beta)) / cfg.phi
    for X, A, is_w in [(ch.W, avg_W, True), (ch.H, avg_H, False)]:
        for idx in np.ndindex(X.shape):
            h = 1e-6
            Xp, Xm = X.copy(), X.copy()
            Xp[idx] += h
            Xm[idx] -= h
            fd = ((full_ll(Xp, ch.H) - full_ll(Xm, ch.H)) if is_w else
                  (full_ll(ch.W, Xp) - full_ll(ch.W, Xm))) / (2 * h)
            assert abs(fd - A[idx]) <= 1e-6 * max(1.0, abs(fd))


# ------------------------------------------------------------------- P7
def test_beta_divergence_special_cases():
    """Section 4: d_2 is half the squared error, beta -> 1 and beta -> 0
    approach the KL and IS divergences, d(v||v) = 0 and mu = v minimises."""
    rng = np.random.default_rng(3)
    for v, mu in rng.gamma(2.0, 1.0, (20, 2)):
        assert oracle.dbeta(v, mu, 2.0) == pytest.approx(0.5 * (v - mu) ** 2, rel=1e-12, abs=1e-15)
        kl = v * np.log(v / mu) - v + mu
        isd = v / mu - np.log(v / mu) - 1
        assert oracle.dbeta(v, mu, 1.0) == pytest.approx(kl, rel=1e-12, abs=1e-15)
        assert oracle.dbeta(v, mu, 0.0) == pytest.approx(isd, rel=1e-12, abs=1e-15)
        assert oracle.dbeta(v, mu, 1.0 + 1e-7) == pytest.approx(kl, rel=1e-5, abs=1e-9)
        assert oracle.dbeta(v, mu, 1e-7) == pytest.approx(isd, rel=1e-5, abs=1e-9)
        for beta in [-1.0, 0.0, 0.5, 1.0, 2.0, 3.0]:
            assert abs(oracle.dbeta(v, v, beta)) < 1e-12
            for d in (0.9, 1.1):
                assert oracle.dbeta(v, v * d, beta) > 0
    assert oracle.dbeta(0.0, 2.5, 1.0) == pytest.approx(2.5)      # 0 log 0 = 0


@pytest.mark.parametrize("beta", BETAS)
def test_loglik_matches_independent_sum(beta):
    wl, cfg, ch = small_problem(beta, "exponential", True, seed=9)
    mu = np.einsum("nk,kn->n", ch.W[wl.row], ch.H[:, wl.col])
    mu = np.maximum(mu, cfg.mu_floor) if beta < 2 else mu
    expect = -np.sum(dbeta_np(wl.val, mu, beta)) / cfg.phi
    assert ch.loglik() == pytest.approx(expect, rel=1e-12)


# ------------------------------------------------------------------- schedule and update form
def test_single_noise_off_step_is_eps_times_drift():
    """Eq. (8)-(9) with the noise removed: x1 = x0 + eps_t * drift_p(x0),
    eps_t = a (t0 + t)^-gamma at the 0-based iteration t, part p = t mod B."""
    wl, cfg, ch = small_problem(2.0, "gaussian", False, seed=4, B=3, I=9, J=8, nnz=40)
    cfg.flags = oracle.FLAG_NOISE_OFF
    cfg.eps_a, cfg.eps_t0, cfg.eps_gamma = 0.02, 3.0, 0.6
    t = 5
    ch.t = t
    dW, dH = ch.drift(t % cfg.B)
    W0, H0 = ch.W.copy(), ch.H.copy()
    ch.run(1)
    eps = 0.02 * (3.0 + t) ** -0.6
    assert cfg.eps(t) == pytest.approx(eps, rel=1e-15)
    np.testing.assert_allclose(ch.W, W0 + eps * dW, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(ch.H, H0 + eps * dH, rtol=1e-13, atol=1e-15)


def test_mirroring_reflects_negative_values():
    """Algorithm 1 / Section 3.2: after the update, x <- |x|."""
    wl, cfg, ch = small_problem(1.0, "exponential", True, seed=6)
    cfg.flags = oracle.FLAG_NOISE_OFF
    cfg.eps_a, cfg.eps_gamma = 5.0, 0.0                  # large step: many go negative
    dW, dH = ch.drift(0)
    W0, H0 = ch.W.copy(), ch.H.copy()
    ch.run(1)
    raw = W0 + 5.0 * dW
    assert (raw < 0).any()
    np.testing.assert_allclose(ch.W, np.abs(raw), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(ch.H, np.abs(H0 + 5.0 * dH), rtol=1e-13, atol=1e-13)


def test_noise_is_sqrt_2eps_times_stream():
    """The injected noise is N(0, 2 eps): with the likelihood and prior
    terms removed (frozen partner, tiny lambda), x1 - x0 - eps*drift equals
    sqrt(2 eps) z with z the documented Philox/Box-Muller stream."""
    wl, cfg, ch = small_problem(2.0, "gaussian", False, seed=8)
    cfg.flags = oracle.FLAG_FREEZE_H
    t = 2
    ch.t = t
    dW, _ = ch.drift(t % cfg.B)
    W0 = ch.W.copy()
    ch.run(1)
    eps = cfg.eps(t)
    for i in range(cfg.I):
        z, _ = oracle.normals(cfg.seed, t, oracle.STREAM_W, i, cfg.K)
        np.testing.assert_allclose(ch.W[i] - W0[i] - eps * dW[i], np.sqrt(2 * eps) * z,
                                   rtol=1e-9, atol=1e-15)


# ------------------------------------------------------------------- P3
@pytest.mark.parametrize("beta,prior,mirror,B", [(2.0, "gaussian", False, 1),
                                                 (2.0, "gaussian", False, 3),
                                                 (1.0, "exponential", True, 1),
                                                 (1.0, "exponential", True, 4)])
def test_noise_off_is_parallel_sgd_with_decreasing_objective(beta, prior, mirror, B):
    """Without noise PSGLD is stratified parallel SGD (the DSGD analogue,
    Section 4.3); at a small constant step the negative log joint falls
    after every cycle of B iterations."""
    wl = workloads.random_sparse(40, 30, 500, 4, B, beta=beta, phi=1.0, prior=prior,
                                 mirror=mirror, data_seed=21, chain_seed=22)
    a = 0.05 * wl.eps_a
    cfg = oracle.Config(I=40, J=30, K=4, B=B, beta=beta, phi=1.0, prior=prior, mirror=mirror,
                        eps_a=a, eps_gamma=0.0, flags=oracle.FLAG_NOISE_OFF)
    ch = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0)

    def neg_log_joint():
        return -(ch.loglik() + log_prior_np(ch.W, ch.H, cfg))

    prev = neg_log_joint()
    for _ in range(30):
        ch.run(B)
        cur = neg_log_joint()
        assert cur < prev
        prev = cur


# ------------------------------------------------------------------- P5
def test_ridge_fixed_point():
    """Gaussian likelihood and prior, H frozen, noise off, B = 1: each w_i
    converges to the ridge solution (lambda I + H_i H_i^T / phi)^-1 H_i v_i / phi,
    checked with numpy.linalg.solve."""
    I, J, K = 8, 12, 3
    rng = np.random.default_rng(31)
    obs = rng.random((I, J)) < 0.6
    row, col = np.nonzero(obs)
    val = rng.normal(2.0, 1.0, len(row))
    W0 = rng.normal(0, 1, (I, K))
    H0 = rng.normal(0, 1, (K, J))
    phi, lam = 0.5, 2.0
    lam_max = max(np.linalg.eigvalsh(lam * np.eye(K) + H0[:, col[row == i]] @ H0[:, col[row == i]].T / phi).max()
                  for i in range(I))
    cfg = oracle.Config(I=I, J=J, K=K, B=1, beta=2.0, phi=phi, prior="gaussian", lambda_w=lam,
                        lambda_h=lam, eps_a=1.0 / lam_max, eps_gamma=0.0,
                        flags=oracle.FLAG_NOISE_OFF | oracle.FLAG_FREEZE_H)
    ch = oracle.Chain(cfg, row, col, val, W0, H0)
    ch.run(4000)
    for i in range(I):
        Hi = H0[:, col[row == i]]
        A = lam * np.eye(K) + Hi @ Hi.T / phi
        b = Hi @ val[row == i] / phi
        np.testing.assert_allclose(ch.W[i], np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)
    np.testing.assert_array_equal(ch.H, H0)


# ------------------------------------------------------------------- P6
def test_ula_gaussian_closed_form():
    """Gaussian likelihood and prior with H frozen, constant step, B = 1:
    each row's chain is the unadjusted Langevin algorithm on the Gaussian
    conditional posterior N(m, Lambda^-1).  Its stationary law is exactly
    N(m, (Lambda - eps Lambda^2 / 2)^-1), which solves
    C = (I - eps Lambda) C (I - eps Lambda) + 2 eps I."""
    I, J, K = 400, 3, 2
    rng = np.random.default_rng(41)
    H0 = np.array([[1.0, 0.5, -0.3], [0.2, 1.1, 0.7]])
    row = np.repeat(np.arange(I), J)
    col = np.tile(np.arange(J), I)
    val = rng.normal(1.0, 1.0, I * J)
    phi, lam = 1.0, 1.0
    Lam = lam * np.eye(K) + H0 @ H0.T / phi
    lmax = np.linalg.eigvalsh(Lam).max()
    eps = 0.5 / lmax
    burn, T = 200, 4200
    cfg = oracle.Config(I=I, J=J, K=K, B=1, beta=2.0, phi=phi, prior="gaussian", lambda_w=lam,
                        lambda_h=lam, eps_a=eps, eps_gamma=0.0, seed=99, burn_in=burn, thin=1,
                        flags=oracle.FLAG_FREEZE_H)
    W0 = rng.normal(0, 1, (I, K))
    ch = oracle.Chain(cfg, row, col, val, W0, H0)
    ch.run(T)
    mW, vW = ch.posterior_mean()[0], ch.posterior_var()[0]
    m_true = np.linalg.solve(Lam, (H0 @ val.reshape(I, J).T / phi)).T       # I x K
    C_ula = np.linalg.inv(Lam - eps * Lam @ Lam / 2)
    C_post = np.linalg.inv(Lam)
    n = T - burn
    # pooled over rows: mean error ~ 0, average variance ~ diag(C_ula)
    tau = 2.0 / (eps * np.linalg.eigvalsh(Lam).min())       # AR(1) integrated time, upper bound
    se_mean = np.sqrt(np.diag(C_ula) * tau / n / I)
    assert np.all(np.abs((mW - m_true).mean(axis=0)) < 5 * se_mean)
    avg_var = vW.mean(axis=0)
    np.testing.assert_allclose(avg_var, np.diag(C_ula), rtol=0.04)
    # and the test separates the ULA law from the exact posterior
    assert np.all(np.abs(np.diag(C_ula) / np.diag(C_post) - 1) > 0.15)


# ------------------------------------------------------------------- bookkeeping
def test_moments_and_heldout_sums_follow_definition():
    """Monte Carlo averages after burn-in (Section 4.2.2): moments of the
    kept samples, and held-out means averaged over the iterations in which
    the cell's block was in the part, evaluated at that iteration's input."""
    wl = workloads.random_sparse(20, 16, 120, 3, 4, beta=1.0, prior="exponential", mirror=True,
                                 data_seed=12, chain_seed=13)
    cfg = oracle.Config(**{k: v for k, v in wl.fit_kwargs().items()})
    cfg.burn_in, cfg.thin = 3, 2
    ch = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
    rp, cp = ch.row_piece, ch.col_piece
    sumW = np.zeros_like(ch.W)
    sumW2 = np.zeros_like(ch.W)
    sumH = np.zeros_like(ch.H)
    ho = np.zeros(len(wl.hrow))
    cnt = np.zeros(len(wl.hrow), dtype=np.int64)
    kept = 0
    for t in range(15):
        if t >= 3:
            inp = part_members(wl.hrow, wl.hcol, rp, cp, cfg.B, t % cfg.B)
            mu = np.einsum("nk,kn->n", ch.W[wl.hrow], ch.H[:, wl.hcol])
            ho[inp] += mu[inp]
            cnt[inp] += 1
        ch.run(1)
        if t >= 3 and (t - 3) % 2 == 0:
            sumW += ch.W
            sumW2 += ch.W ** 2
            sumH += ch.H
            kept += 1
    assert ch.n_kept == kept == 6
    np.testing.assert_allclose(ch.sumW, sumW, rtol=1e-14)
    np.testing.assert_allclose(ch.sumW2, sumW2, rtol=1e-14)
    np.testing.assert_allclose(ch.sumH, sumH, rtol=1e-14)
    np.testing.assert_array_equal(ch.ho_cnt, cnt)
    np.testing.assert_allclose(ch.ho_sum, ho, rtol=1e-13)
    mW, _ = ch.posterior_mean()
    vW, _ = ch.posterior_var()
    np.testing.assert_allclose(mW, sumW / kept, rtol=1e-14)
    np.testing.assert_allclose(vW, sumW2 / kept - (sumW / kept) ** 2, rtol=1e-10, atol=1e-14)


def test_resume_is_bit_identical():
    """The noise is keyed by (seed, t, stream, index, k), so stopping and
    resuming the chain changes nothing."""
    wl = workloads.random_sparse(30, 25, 200, 5, 3, data_seed=2, chain_seed=3)
    cfg = oracle.Config(**wl.fit_kwargs())
    cfg.burn_in = 2
    a = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
    a.run(10)
    b = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
    b.run(4)
    c = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
    c.set_state(b.W, b.H, b.t)
    c.sumW, c.sumW2, c.sumH, c.sumH2 = b.sumW.copy(), b.sumW2.copy(), b.sumH.copy(), b.sumH2.copy()
    c.n_kept, c.ho_sum, c.ho_cnt = b.n_kept, b.ho_sum.copy(), b.ho_cnt.copy()
    c.run(6)
    for x, y in [(a.W, c.W), (a.H, c.H), (a.sumW, c.sumW), (a.sumH2, c.sumH2), (a.ho_sum, c.ho_sum)]:
        assert np.array_equal(x, y)


# ------------------------------------------------- Condition 2: random part order
def _skewed_chain(order, seed=3):
    """B = 4 pieces chosen so the four parts hold very different numbers of
    entries (one of them none)."""
    I, J, K, B = 12, 12, 2, 4
    rp = np.repeat(np.arange(B), 3).astype(np.int32)
    cp = rp.copy()
    rng = np.random.default_rng(seed)
    want = {0: 30, 1: 12, 2: 0, 3: 6}        # entries per part
    row, col = [], []
    for p, n in want.items():
        cells = [(i, j) for i in range(I) for j in range(J) if (rp[i] + p) % B == cp[j]]
        pick = rng.choice(len(cells), size=n, replace=False)
        row += [cells[k][0] for k in pick]
        col += [cells[k][1] for k in pick]
    row, col = np.array(row, np.int32), np.array(col, np.int32)
    val = rng.gamma(2.0, 1.0, len(row))
    W0, H0 = rng.gamma(2.0, 0.5, (I, K)), rng.gamma(2.0, 0.5, (K, J))
    cfg = oracle.Config(I=I, J=J, K=K, B=B, beta=2.0, phi=1.0, eps_a=1e-2, eps_gamma=0.0, seed=77,
                        flags=oracle.FLAG_NOISE_OFF | oracle.FLAG_FREEZE_H, part_order=order)
    return oracle.Chain(cfg, row, col, val, W0, H0, row_piece=rp, col_piece=cp), row, col, val, W0, H0, cfg, rp, cp


def test_random_part_frequencies_follow_condition2():
    """Condition 2: p(Pi) = |Pi| / N.  Over many iterations the drawn parts'
    frequencies match n_p / N (chi-square), and the empty part never occurs."""
    ch = _skewed_chain("random")[0]
    n_p = ch.part_sizes()
    assert list(n_p) == [30, 12, 0, 6]
    draws = np.array([ch.part_at(t) for t in range(60_000)])
    cnt = np.bincount(draws, minlength=4)
    assert cnt[2] == 0
    expected = n_p / n_p.sum() * len(draws)
    m = expected > 0
    chi2 = float(np.sum((cnt[m] - expected[m]) ** 2 / expected[m]))
    assert chi2 < 16.3, (cnt, expected)    # 3 degrees of freedom, p < 0.001
    # the cyclic order is t mod B
    cyc = _skewed_chain("cyclic")[0]
    assert [cyc.part_at(t) for t in range(9)] == [t % 4 for t in range(9)]


def test_random_order_steps_use_the_drawn_part():
    """A noise-off step at iteration t depends exactly on the entries of the
    part drawn for t: perturbing an entry changes W iff it lies in that part."""
    ch0, row, col, val, W0, H0, cfg, rp, cp = _skewed_chain("random")
    for t in range(6):
        p = ch0.part_at(t)
        base = oracle.Chain(cfg, row, col, val, W0, H0, row_piece=rp, col_piece=cp)
        base.t = t
        base.run(1)
        for e in range(len(row)):
            v2 = val.copy()
            v2[e] += 1.0
            ch = oracle.Chain(cfg, row, col, v2, W0, H0, row_piece=rp, col_piece=cp)
            ch.t = t
            ch.run(1)
            inside = (rp[row[e]] + p) % 4 == cp[col[e]]
            assert (not np.array_equal(ch.W, base.W)) == inside, (t, e)


# ------------------------------------------------------------------- P9
def test_results_do_not_depend_on_the_thread_count():
    """The oracle sums each block of a part on one thread, in (i, j) order,
    and steps rows and columns independently, so a run on one thread and on
    several gives the same bits (factors, moments, held-out sums, bounds).
    The problem is large enough that every parallel loop does fork."""
    wl = workloads.random_sparse(4000, 2500, 60_000, 16, 5, beta=1.0, prior="exponential", mirror=True,
                                 zipf_a=1.0, data_seed=61, chain_seed=62, burn_in=2, thin=2)
    threads0 = oracle.threads()
    runs = []
    try:
        for n in (1, 3, 8):
            oracle.threads(n)
            assert oracle.threads() == n
            cfg = oracle.Config(**wl.fit_kwargs())
            ch = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
            ch.run(6)
            bW, bH = ch.run(1, bounds=True)
            runs.append((ch.W, ch.H, ch.sumW, ch.sumH2, ch.ho_sum, bW, bH))
    finally:
        oracle.threads(threads0)
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            assert np.array_equal(a, b)
