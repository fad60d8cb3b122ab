"""Pin of the oracle's single-step tolerance scale c_x.

Every single-step parity verdict divides |x_gpu - x_ref| by the oracle's
per-parameter scale
    c_x = |x_old| + eps (s_p G+_x + |prior'(x_old)|) + sigma R_x,
the magnitude of every term of the Langevin step of Eq. (8)-(9) that an FP32
evaluation rounds: G+ is the sum over the block's entries of the absolute
values of the gradient's terms, (|v| + sum_k' |w_ik' h_k'j|) mu~^(beta-2)/phi
times |partner|, and R_x the Box-Muller radius of x's normal.  The numpy code
here recomputes c_x from that definition without calling the oracle's
gradient or bound code; the radius is recovered from the normal pair it
produced (r^2 = z_2m^2 + z_2m+1^2 for the two outputs of one Box-Muller
transform), so a mistake in how the oracle assembles c_x (a swapped |w| and
|h|, a dropped eps, a missing sigma R term) fails here.
"""
import numpy as np
import pytest

import oracle
import workloads


def radii(seed, t, stream, index, K):
    """Box-Muller radius of each of the K normals of one row/column, from the
    normal pairs (the stream is drawn in whole quads, so K is rounded up)."""
    K4 = (K + 3) // 4 * 4
    z, _ = oracle.normals(seed, t, stream, index, K4)
    pair = np.sqrt(z[0::2] ** 2 + z[1::2] ** 2)
    return np.repeat(pair, 2)[:K]


def c_x_numpy(wl, cfg, W, H, t, rp, cp, noise=True):
    """(c_W, c_H) of the step from iteration t, from the definition."""
    B = cfg.B
    p = t % B
    eps = cfg.eps_a * (cfg.eps_t0 + t) ** (-cfg.eps_gamma)
    sigma = np.sqrt(2.0 * eps)
    inpart = (rp[wl.row] + p) % B == cp[wl.col]
    N, n_p = len(wl.row), int(inpart.sum())
    s_p = N / n_p if n_p else 0.0
    r, c, v = wl.row[inpart], wl.col[inpart], wl.val[inpart].astype(np.float64)
    Wm = np.abs(W) if cfg.mirror else W
    Hm = np.abs(H) if cfg.mirror else H
    mu = np.einsum("nk,kn->n", Wm[r], Hm[:, c])
    mu_abs = np.einsum("nk,kn->n", np.abs(W[r]), np.abs(H[:, c]))
    mu_t = np.maximum(mu, cfg.mu_floor) if cfg.beta < 2 else mu
    e_abs = (np.abs(v) + mu_abs) * mu_t ** (cfg.beta - 2.0) / cfg.phi
    Gw = np.zeros_like(W)
    Gh = np.zeros_like(H)
    np.add.at(Gw, r, e_abs[:, None] * np.abs(H[:, c]).T)
    np.add.at(Gh.T, c, e_abs[:, None] * np.abs(W[r]))
    if cfg.prior == "exponential":
        pw, ph = np.full_like(W, cfg.lambda_w), np.full_like(H, cfg.lambda_h)
    else:
        pw, ph = cfg.lambda_w * np.abs(W), cfg.lambda_h * np.abs(H)
    Rw = np.zeros_like(W)
    Rh = np.zeros_like(H)
    if noise:
        for i in range(cfg.I):
            Rw[i] = radii(cfg.seed, t, oracle.STREAM_W, i, cfg.K)
        for j in range(cfg.J):
            Rh[:, j] = radii(cfg.seed, t, oracle.STREAM_H, j, cfg.K)
    cW = np.abs(W) + eps * (s_p * Gw + pw) + sigma * Rw
    cH = np.abs(H) + eps * (s_p * Gh + ph) + sigma * Rh
    return cW, cH, dict(eps=eps, sigma=sigma, s_p=s_p, Gw=Gw, Gh=Gh, Rw=Rw, Rh=Rh, pw=pw, ph=ph)


CASES = [
    # beta, prior, mirror, flags, t
    (2.0, "gaussian", False, 0, 0),
    (2.0, "gaussian", False, 0, 5),
    (1.0, "exponential", True, 0, 3),
    (0.5, "exponential", True, 0, 2),
    (0.0, "gaussian", True, 0, 4),
    (1.0, "exponential", True, oracle.FLAG_NOISE_OFF, 1),
]


def make_chain(beta, prior, mirror, flags, seed=21):
    wl = workloads.random_sparse(23, 17, 160, 6, 3, beta=beta, phi=0.8, prior=prior, mirror=mirror,
                                 data_seed=seed, chain_seed=seed + 1, zipf_a=1.0)
    cfg = oracle.Config(**wl.fit_kwargs())
    cfg.flags = flags
    cfg.lambda_w, cfg.lambda_h = 1.3, 0.7
    ch = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0)
    return wl, cfg, ch


@pytest.mark.parametrize("beta,prior,mirror,flags,t", CASES)
def test_bound_equals_its_definition(beta, prior, mirror, flags, t):
    wl, cfg, ch = make_chain(beta, prior, mirror, flags)
    ch.run(t)                                  # a state that is not the starting point
    W, H = ch.W.copy(), ch.H.copy()
    bW, bH = ch.run(1, bounds=True)
    cW, cH, _ = c_x_numpy(wl, cfg, W, H, t, ch.row_piece, ch.col_piece,
                          noise=not (flags & oracle.FLAG_NOISE_OFF))
    np.testing.assert_allclose(bW, cW, rtol=1e-12, atol=0)
    np.testing.assert_allclose(bH, cH, rtol=1e-12, atol=0)


def test_planted_bound_mistakes_are_caught():
    """Each plausible slip in assembling c_x moves it far beyond the 1e-12
    agreement the pin demands: a missing sigma R term, the partner's |h|
    swapped for the item's own |w|, a dropped eps, the part scale left out."""
    wl, cfg, ch = make_chain(2.0, "gaussian", False, 0)
    ch.run(2)
    W, H = ch.W.copy(), ch.H.copy()
    bW, bH = ch.run(1, bounds=True)
    cW, cH, d = c_x_numpy(wl, cfg, W, H, 2, ch.row_piece, ch.col_piece)
    z = np.zeros_like(W)
    for i in range(cfg.I):
        z[i], _ = oracle.normals(cfg.seed, 2, oracle.STREAM_W, i, cfg.K)
    mutants = {
        "no sigma R": np.abs(W) + d["eps"] * (d["s_p"] * d["Gw"] + d["pw"]),
        "no eps": np.abs(W) + (d["s_p"] * d["Gw"] + d["pw"]) + d["sigma"] * d["Rw"],
        "no part scale": np.abs(W) + d["eps"] * (d["Gw"] + d["pw"]) + d["sigma"] * d["Rw"],
        "sigma |z| for sigma R": np.abs(W) + d["eps"] * (d["s_p"] * d["Gw"] + d["pw"]) + d["sigma"] * np.abs(z),
    }
    # the item's own |w| in place of the partner's |h| inside G+
    p = 2 % cfg.B
    r, c, v = wl.row, wl.col, wl.val.astype(np.float64)
    inpart = (ch.row_piece[r] + p) % cfg.B == ch.col_piece[c]
    mu_abs = np.einsum("nk,kn->n", np.abs(W[r[inpart]]), np.abs(H[:, c[inpart]]))
    e_abs = (np.abs(v[inpart]) + mu_abs) / cfg.phi          # beta = 2: no power of mu
    Gswap = np.zeros_like(W)
    np.add.at(Gswap, r[inpart], e_abs[:, None] * np.abs(W[r[inpart]]))
    mutants["|w| for |h|"] = np.abs(W) + d["eps"] * (d["s_p"] * Gswap + d["pw"]) + d["sigma"] * d["Rw"]
    np.testing.assert_allclose(bW, cW, rtol=1e-12, atol=0)
    for name, m in mutants.items():
        rel = np.max(np.abs(m - bW) / bW)
        assert rel > 1e-6, (name, rel)


def test_tolerance_separates_rounding_from_a_wrong_step():
    """With the true c_x, an FP32-like rounding of every term of the step
    (relative 2^-24 of each magnitude) scores far below the 1e-5 bar, while
    a wrong step -- the noise term's sign flipped on one parameter -- scores
    far above it."""
    wl, cfg, ch = make_chain(1.0, "exponential", True, 0)
    ch.run(3)
    W, H = ch.W.copy(), ch.H.copy()
    bW, _ = ch.run(1, bounds=True)
    _, _, d = c_x_numpy(wl, cfg, W, H, 3, ch.row_piece, ch.col_piece)
    ulp = 2.0 ** -24
    rounding = ulp * (np.abs(W) + d["eps"] * (d["s_p"] * d["Gw"] + d["pw"]) + d["sigma"] * d["Rw"])
    assert np.max(rounding / bW) < 1e-6
    z = np.zeros_like(W)
    for i in range(cfg.I):
        z[i], _ = oracle.normals(cfg.seed, 3, oracle.STREAM_W, i, cfg.K)
    k = np.unravel_index(np.argmax(np.abs(z)), z.shape)
    wrong = np.zeros_like(W)
    wrong[k] = 2.0 * d["sigma"] * abs(z[k])
    assert np.max(wrong / bW) > 1e-2
