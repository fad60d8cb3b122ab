"""Seeded synthetic workloads shaped like the paper's experiments.

These generators feed both the GPU library and the FP64 oracle; they hold
none of the sampler's arithmetic (no gradients, no noise stream, no update).
Every array is drawn with ``numpy.random.default_rng(seed)`` so a workload is
reproducible on any machine with the same numpy.

The paper's own data (a piano recording, the MovieLens 10M ratings) is not
available, so synthetic stand-ins of the same shape and value range are used:
  * ``dense_poisson``   -- Poisson NMF on a dense matrix (Section 4.2.1 setup).
  * ``sparse_ratings``  -- recommender-shaped ratings 1..5: lognormal row
    activity, Zipf column popularity drawn without replacement per row
    (stands in for MovieLens 10M, Section 4.3).
  * ``dense_tweedie``   -- spectrogram-shaped non-negative matrix with
    compound Poisson-gamma (Tweedie, beta = 0.5) noise (Sections 4.2.1-4.2.2).
  * ``serving_job``     -- one job of a stream of mixed-size factorisation
    jobs, with ``job_arrivals`` giving Poisson arrival times.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Workload:
    name: str
    I: int
    J: int
    K: int
    B: int
    beta: float
    phi: float
    prior: str
    lambda_w: float
    lambda_h: float
    mirror: bool
    eps_a: float
    eps_t0: float
    eps_gamma: float
    seed: int
    T: int
    burn_in: int
    thin: int
    row: np.ndarray          # training entries (int32, int32, float32)
    col: np.ndarray
    val: np.ndarray
    hrow: np.ndarray         # held-out cells
    hcol: np.ndarray
    hval: np.ndarray
    W0: np.ndarray           # I x K float32
    H0: np.ndarray           # K x J float32
    dense: Optional[np.ndarray] = None   # I x J float32 when the matrix is dense
    mask: Optional[np.ndarray] = None    # I x J uint8, 1 = training cell
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(len(self.row))

    def fit_kwargs(self) -> dict:
        """Model / schedule settings shared by the oracle and the library."""
        return dict(I=self.I, J=self.J, K=self.K, B=self.B, beta=self.beta, phi=self.phi,
                    prior=self.prior, lambda_w=self.lambda_w, lambda_h=self.lambda_h,
                    mirror=self.mirror, eps_a=self.eps_a, eps_t0=self.eps_t0,
                    eps_gamma=self.eps_gamma, seed=self.seed, burn_in=self.burn_in,
                    thin=self.thin)


# --------------------------------------------------------------------- helpers
def init_factors(rng, I, J, K, vbar, mirror):
    """Starting point: every element near sqrt(vbar/K), so that w_i . h_j
    starts near the mean observed value, with 10% multiplicative jitter."""
    s = np.sqrt(max(vbar, 1e-3) / K)
    W0 = s * (1.0 + 0.1 * rng.standard_normal((I, K)))
    H0 = s * (1.0 + 0.1 * rng.standard_normal((K, J)))
    if mirror:
        W0, H0 = np.abs(W0), np.abs(H0)
    return W0.astype(np.float32), H0.astype(np.float32)


def step_scale(row, col, val, I, J, beta, phi):
    """Step-size constant a = 0.5 / L, with L a curvature estimate of the
    heaviest row or column: n_max * max(vbar, 1)^(beta - 1) / phi."""
    n_max = max(int(np.bincount(row, minlength=I).max(initial=0)),
                int(np.bincount(col, minlength=J).max(initial=0)), 1)
    vbar = float(np.mean(val)) if len(val) else 1.0
    L = n_max * max(vbar, 1.0) ** (beta - 1.0) / phi
    return 0.5 / L


def _split_heldout(rng, n, frac):
    n_ho = int(round(frac * n))
    perm = rng.permutation(n)
    return np.sort(perm[n_ho:]), np.sort(perm[:n_ho])


def gaussian_factor_moments(K_true, mean_dot=3.5, sd_dot=1.0):
    """(m, s^2) of iid N(m, s^2) factor elements such that w . h over K_true
    terms has the given mean and standard deviation."""
    m = np.sqrt(mean_dot / K_true)
    s2 = -m * m + np.sqrt(m ** 4 + sd_dot ** 2 / K_true)
    return m, s2


def zipf_columns_without_replacement(rng, counts, J, a):
    """For each row r draw counts[r] distinct columns, the column of popularity
    rank q having weight q^-a; rank -> column id is a random permutation.
    Sampling is successive (weighted, without replacement).  Light rows:
    draw with replacement and keep the first counts[r] distinct columns in
    draw order, topping up only the rows still short.  Rows asking for more
    than J/16 columns: Gumbel-top-k, which samples the same law exactly.
    Returns (row, col) sorted by (row, col)."""
    counts = np.asarray(counts, dtype=np.int64)
    I = len(counts)
    w = np.arange(1, J + 1, dtype=np.float64) ** (-a)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    rank_to_col = rng.permutation(J).astype(np.int64)
    heavy = counts > max(J // 16, 1)
    done = []
    # pending rows: distinct keys so far, in draw order within each row
    pend_rows = np.nonzero(~heavy)[0]
    pend_keys = np.zeros(0, dtype=np.int64)
    for _ in range(200):
        if len(pend_rows) == 0:
            break
        have = np.bincount(pend_keys // J, minlength=I)[pend_rows]
        need = counts[pend_rows] - have
        over = np.ceil(need * 1.25).astype(np.int64) + 4
        r = np.repeat(pend_rows, over)
        c = rank_to_col[np.minimum(np.searchsorted(cdf, rng.random(len(r))), J - 1)]
        cat = np.concatenate([pend_keys, r * J + c])
        _, first = np.unique(cat, return_index=True)
        first.sort()
        keys = cat[first]                           # distinct, in draw order
        rows_k = keys // J
        order = np.argsort(rows_k, kind="stable")   # group by row, keep draw order
        keys, rows_k = keys[order], rows_k[order]
        start = np.searchsorted(rows_k, rows_k, side="left")
        pos = np.arange(len(keys)) - start
        keys = keys[pos < counts[rows_k]]
        rows_k = keys // J
        got = np.bincount(rows_k, minlength=I)
        finished = got >= counts
        fin_mask = finished[rows_k]
        done.append(keys[fin_mask])
        pend_keys = keys[~fin_mask]
        pend_rows = pend_rows[~finished[pend_rows]]
    else:
        raise RuntimeError("column sampling did not converge")
    logw = np.log(w)
    hv = np.nonzero(heavy)[0]
    chunk = max(1, (1 << 24) // J)
    for s in range(0, len(hv), chunk):
        rows = hv[s:s + chunk]
        g = logw[None, :] - np.log(-np.log(rng.random((len(rows), J))))
        for m, r in enumerate(rows):
            top = np.argpartition(-g[m], counts[r] - 1)[: counts[r]]
            done.append(r * J + rank_to_col[top])
    keys = np.sort(np.concatenate(done))
    return (keys // J).astype(np.int32), (keys % J).astype(np.int32)


def lognormal_row_counts(rng, I, J, total, mu=4.0, sigma=1.2):
    """Row activity: x_i ~ LN(mu, sigma), rescaled to sum to `total`, each
    count clipped to [1, J]; the rounding residue is spread one by one."""
    x = rng.lognormal(mu, sigma, I)
    n = np.clip(np.round(x * total / x.sum()), 1, J).astype(np.int64)
    diff = int(total - n.sum())
    order = rng.permutation(I)
    k = 0
    while diff != 0:
        r = order[k % I]
        if diff > 0 and n[r] < J:
            n[r] += 1
            diff -= 1
        elif diff < 0 and n[r] > 1:
            n[r] -= 1
            diff += 1
        k += 1
    return n


# ------------------------------------------------------------------ workloads
def dense_poisson(I=256, J=256, K=8, B=4, heldout=0.1, data_seed=1001, chain_seed=2001,
                  T=200, burn_in=100, thin=1, eps_a=1e-3, eps_t0=1.0, eps_gamma=0.51,
                  name="dense_poisson_256"):
    """Poisson NMF: W*, H* ~ Gamma(1, 1), v_ij ~ Poisson((W*H*)_ij), a fraction
    of the cells held out uniformly; exponential priors of rate 1, mirroring."""
    rng = np.random.default_rng(data_seed)
    Wt = rng.gamma(1.0, 1.0, (I, K))
    Ht = rng.gamma(1.0, 1.0, (K, J))
    V = rng.poisson(Wt @ Ht).astype(np.float32)
    cells = I * J
    tr, ho = _split_heldout(rng, cells, heldout)
    mask = np.zeros(cells, dtype=np.uint8)
    mask[tr] = 1
    mask = mask.reshape(I, J)
    row, col = (tr // J).astype(np.int32), (tr % J).astype(np.int32)
    hrow, hcol = (ho // J).astype(np.int32), (ho % J).astype(np.int32)
    val = V.reshape(-1)[tr]
    hval = V.reshape(-1)[ho]
    W0, H0 = init_factors(np.random.default_rng(chain_seed), I, J, K, float(val.mean()), True)
    return Workload(name, I, J, K, B, 1.0, 1.0, "exponential", 1.0, 1.0, True,
                    eps_a, eps_t0, eps_gamma, chain_seed, T, burn_in, thin,
                    row, col, val, hrow, hcol, hval, W0, H0, dense=V, mask=mask)


def sparse_ratings(I=70_000, J=10_700, nnz=10_000_000, K_true=20, K=50, B=32, zipf_a=1.0,
                   heldout=0.1, noise_sd=0.5, data_seed=1002, chain_seed=2002, T=1000,
                   burn_in=500, thin=1, name="sparse_ratings_70k"):
    """Recommender-shaped ratings: lognormal(4, 1.2) row activity, Zipf column
    popularity without replacement per row, v = round(clip(w.h + noise, 1, 5))
    from rank-K_true Gaussian factors; Gaussian likelihood with
    phi = noise variance + rounding variance, Gaussian priors, no mirroring."""
    rng = np.random.default_rng(data_seed)
    counts = lognormal_row_counts(rng, I, J, nnz)
    r_all, c_all = zipf_columns_without_replacement(rng, counts, J, zipf_a)
    m, s2 = gaussian_factor_moments(K_true)
    Wt = (m + np.sqrt(s2) * rng.standard_normal((I, K_true))).astype(np.float32)
    Ht = (m + np.sqrt(s2) * rng.standard_normal((J, K_true))).astype(np.float32)
    v = np.empty(len(r_all), dtype=np.float32)
    chunk = 1 << 22
    for s in range(0, len(r_all), chunk):
        e = slice(s, s + chunk)
        dot = np.einsum("nk,nk->n", Wt[r_all[e]], Ht[c_all[e]])
        v[e] = np.round(np.clip(dot + noise_sd * rng.standard_normal(len(dot)), 1, 5))
    tr, ho = _split_heldout(rng, len(r_all), heldout)
    row, col, val = r_all[tr], c_all[tr], v[tr]
    hrow, hcol, hval = r_all[ho], c_all[ho], v[ho]
    phi = noise_sd ** 2 + 1.0 / 12.0
    a = step_scale(row, col, val, I, J, 2.0, phi)
    W0, H0 = init_factors(np.random.default_rng(chain_seed), I, J, K, float(val.mean()), False)
    return Workload(name, I, J, K, B, 2.0, phi, "gaussian", 1.0, 1.0, False,
                    a, 1.0, 0.51, chain_seed, T, burn_in, thin,
                    row, col, val, hrow, hcol, hval, W0, H0,
                    meta=dict(zipf_a=zipf_a, K_true=K_true, nnz_total=int(len(r_all))))


def dense_tweedie(I=1025, J=100_000, K_true=64, K=64, B=16, heldout=0.1, data_seed=1003,
                  chain_seed=2003, T=1000, burn_in=500, thin=1, name="dense_tweedie_1025x100k"):
    """Spectrogram-shaped non-negative matrix: W* ~ Gamma(2, 1), H* ~ Gamma(0.5, 1),
    v ~ compound Poisson-gamma Tweedie with power 1.5 (beta = 2 - 1.5 = 0.5) and
    phi = 1: v = sum of Pois(2 sqrt(mu)) exponentials of mean sqrt(mu)/2.
    Fit with beta = 0.5, exponential priors, mirroring."""
    rng = np.random.default_rng(data_seed)
    Wt = rng.gamma(2.0, 1.0, (I, K_true)).astype(np.float32)
    Ht = rng.gamma(0.5, 1.0, (K_true, J)).astype(np.float32)
    V = compound_poisson_matrix(rng, Wt, Ht)
    cells = I * J
    tr, ho = _split_heldout(rng, cells, heldout)
    mask = np.zeros(cells, dtype=np.uint8)
    mask[tr] = 1
    mask = mask.reshape(I, J)
    row, col = (tr // J).astype(np.int32), (tr % J).astype(np.int32)
    hrow, hcol = (ho // J).astype(np.int32), (ho % J).astype(np.int32)
    flat = V.reshape(-1)
    val, hval = flat[tr], flat[ho]
    a = step_scale(row, col, val, I, J, 0.5, 1.0)
    W0, H0 = init_factors(np.random.default_rng(chain_seed), I, J, K, float(val.mean()), True)
    return Workload(name, I, J, K, B, 0.5, 1.0, "exponential", 1.0, 1.0, True,
                    a, 1.0, 0.51, chain_seed, T, burn_in, thin,
                    row, col, val, hrow, hcol, hval, W0, H0, dense=V, mask=mask)


def compound_poisson_matrix(rng, Wt, Ht):
    """V ~ TW(mu = Wt Ht, phi = 1, beta = 0.5): the Tweedie law of power
    p = 2 - beta = 1.5 is a compound Poisson-gamma, v = sum of N ~ Pois(2
    sqrt(mu)) gamma variables of shape 1 and scale sqrt(mu) / 2 (v = 0 when
    N = 0), drawn a few million cells at a time."""
    I, J = Wt.shape[0], Ht.shape[1]
    V = np.empty((I, J), dtype=np.float32)
    rows_per = max(1, (1 << 22) // J)
    for r0 in range(0, I, rows_per):
        mu = (Wt[r0:r0 + rows_per].astype(np.float64) @ Ht.astype(np.float64))
        sq = np.sqrt(mu)
        n = rng.poisson(2.0 * sq)
        g = rng.gamma(np.maximum(n, 1), 0.5 * sq)
        V[r0:r0 + rows_per] = np.where(n > 0, g, 0.0)
    return V


def paper_compound_poisson(I=1024, J=1024, K=32, B=32, data_seed=1013, chain_seed=2013, T=10_000,
                           burn_in=5_000, thin=10, name="paper_cpoisson_1024"):
    """The paper's compound Poisson experiment (Section 4.2.1): W, H drawn
    from the model's exponential priors (rate 1), V ~ TW(WH, phi = 1,
    beta = 0.5), every cell observed; fit with the same model (exponential
    priors, mirroring), K = 32, B = I / 32."""
    rng = np.random.default_rng(data_seed)
    Wt = rng.gamma(1.0, 1.0, (I, K)).astype(np.float32)
    Ht = rng.gamma(1.0, 1.0, (K, J)).astype(np.float32)
    V = compound_poisson_matrix(rng, Wt, Ht)
    row, col = np.nonzero(np.ones((I, J), dtype=bool))
    row, col = row.astype(np.int32), col.astype(np.int32)
    val = V.reshape(-1)
    empty = np.zeros(0, dtype=np.int32)
    a = step_scale(row, col, val, I, J, 0.5, 1.0)
    W0, H0 = init_factors(np.random.default_rng(chain_seed), I, J, K, float(val.mean()), True)
    return Workload(name, I, J, K, B, 0.5, 1.0, "exponential", 1.0, 1.0, True,
                    a, 1.0, 0.51, chain_seed, T, burn_in, thin,
                    row, col, val, empty, empty, np.zeros(0, dtype=np.float32), W0, H0,
                    dense=V, mask=np.ones((I, J), dtype=np.uint8))


def random_sparse(I, J, nnz, K, B, beta=2.0, phi=1.0, prior="gaussian", mirror=False,
                  data_seed=7, chain_seed=8, heldout=0.1, eps_a=None, T=10, burn_in=0, thin=1,
                  zipf_a=None, name="random_sparse"):
    """Small problems for parity tests: uniform or Zipf-skewed support,
    values from a low-rank non-negative model (so every beta is valid)."""
    rng = np.random.default_rng(data_seed)
    total = int(round(nnz / (1.0 - heldout)))
    total = min(total, I * J)
    if zipf_a is None:
        keys = np.sort(rng.choice(I * J, size=total, replace=False))
        r_all, c_all = (keys // J).astype(np.int32), (keys % J).astype(np.int32)
    else:
        counts = lognormal_row_counts(rng, I, J, total, 2.0, 1.0)
        r_all, c_all = zipf_columns_without_replacement(rng, counts, J, zipf_a)
    Kt = max(2, K // 2)
    Wt = rng.gamma(1.0, 1.0, (I, Kt))
    Ht = rng.gamma(1.0, 1.0, (J, Kt))
    mu = np.einsum("nk,nk->n", Wt[r_all], Ht[c_all])
    v = (mu * rng.gamma(4.0, 0.25, len(mu)) + 0.05).astype(np.float32)
    tr, ho = _split_heldout(rng, len(r_all), heldout)
    row, col, val = r_all[tr], c_all[tr], v[tr]
    hrow, hcol, hval = r_all[ho], c_all[ho], v[ho]
    a = eps_a if eps_a is not None else step_scale(row, col, val, I, J, beta, phi)
    W0, H0 = init_factors(np.random.default_rng(chain_seed), I, J, K, float(val.mean()), mirror)
    return Workload(name, I, J, K, B, beta, phi, prior, 1.0, 1.0, mirror,
                    a, 1.0, 0.51, chain_seed, T, burn_in, thin,
                    row, col, val, hrow, hcol, hval, W0, H0)


def to_dense(wl: Workload):
    """Dense I x J value matrix and training mask of a sparse workload."""
    V = np.zeros((wl.I, wl.J), dtype=np.float32)
    mask = np.zeros((wl.I, wl.J), dtype=np.uint8)
    V[wl.row, wl.col] = wl.val
    V[wl.hrow, wl.hcol] = wl.hval
    mask[wl.row, wl.col] = 1
    return V, mask


def serving_job(j, seed0=5000, T=500, burn_in=250, thin=10, heldout=0.1, max_side=4096, name="serving_job"):
    """Job j of the serving stream: I, J log-uniform on [64, max_side], observed
    density log-uniform on [0.01, 1] (uniform support), K from {8, 16, 32, 64},
    and either Poisson NMF data (Gamma(1, 1) factors of rank K, v ~ Poisson,
    fit with beta = 1, exponential priors, mirroring) or Gaussian data (rank-K
    Gaussian factors with w.h of mean 3.5 and sd 1, v = w.h + N(0, 0.5^2),
    fit with beta = 2, phi = 0.25, Gaussian priors).  B = clamp(min(I, J) //
    128, 1, 32).  Dense jobs (density > 0.3) carry V and the training mask."""
    rng = np.random.default_rng(seed0 + j)
    lo, hi = np.log(64.0), np.log(float(max_side))
    I = int(round(np.exp(rng.uniform(lo, hi))))
    J = int(round(np.exp(rng.uniform(lo, hi))))
    rho = float(np.exp(rng.uniform(np.log(0.01), 0.0)))
    K = int(rng.choice([8, 16, 32, 64]))
    poisson = bool(rng.integers(0, 2))
    B = int(min(32, max(1, min(I, J) // 128)))
    cells = I * J
    n_obs = max(2, int(round(rho * cells)))
    keys = np.sort(rng.choice(cells, size=n_obs, replace=False))
    if poisson:
        Wt = rng.gamma(1.0, 1.0, (I, K)).astype(np.float32)
        Ht = rng.gamma(1.0, 1.0, (K, J)).astype(np.float32)
    else:
        m, s2 = gaussian_factor_moments(K)
        Wt = (m + np.sqrt(s2) * rng.standard_normal((I, K))).astype(np.float32)
        Ht = (m + np.sqrt(s2) * rng.standard_normal((K, J))).astype(np.float32)
    mu = (Wt @ Ht).reshape(-1)[keys].astype(np.float64)
    if poisson:
        v = rng.poisson(mu).astype(np.float32)
        beta, phi, prior, mirror = 1.0, 1.0, "exponential", True
    else:
        v = (mu + 0.5 * rng.standard_normal(len(mu))).astype(np.float32)
        beta, phi, prior, mirror = 2.0, 0.25, "gaussian", False
    tr, ho = _split_heldout(rng, n_obs, heldout)
    rk, ck = (keys // J).astype(np.int32), (keys % J).astype(np.int32)
    row, col, val = rk[tr], ck[tr], v[tr]
    hrow, hcol, hval = rk[ho], ck[ho], v[ho]
    a = step_scale(row, col, val, I, J, beta, phi)
    W0, H0 = init_factors(np.random.default_rng(seed0 + 10_000 + j), I, J, K,
                          float(val.mean()) if len(val) else 1.0, mirror)
    dense = mask = None
    if rho > 0.3:
        dense = np.zeros((I, J), dtype=np.float32)
        mask = np.zeros((I, J), dtype=np.uint8)
        dense[row, col] = val
        dense[hrow, hcol] = hval
        mask[row, col] = 1
    return Workload(f"{name}_{j}", I, J, K, B, beta, phi, prior, 1.0, 1.0, mirror,
                    a, 1.0, 0.51, seed0 + 20_000 + j, T, burn_in, thin,
                    row, col, val, hrow, hcol, hval, W0, H0, dense=dense, mask=mask,
                    meta=dict(density=rho, poisson=poisson))


def job_arrivals(n_jobs, rate=20.0, seed=3005):
    """Arrival times (seconds) of a Poisson process of the given rate; rate
    0 means every job arrives at time 0."""
    if rate <= 0:
        return np.zeros(n_jobs)
    return np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, n_jobs))


# ------------------------------------------------------------- named configs
def by_name(name):
    """The named workloads the benchmark, the long-run parity tests and the
    stored oracle results share (moments kept every 10th post-burn-in
    iteration where the run is 1000 iterations long)."""
    if name == "dense_poisson_256":
        return dense_poisson()
    if name == "sparse_ratings_70k":
        wl = sparse_ratings()
    elif name == "dense_tweedie_1025x100k":
        wl = dense_tweedie()
    elif name == "sparse_ratings_480k":
        wl = sparse_ratings(I=480_000, J=17_800, nnz=100_000_000, K_true=30, K=100, B=64, zipf_a=1.1,
                            data_seed=1004, chain_seed=2004, name=name)
    elif name == "sparse_ratings_small":
        wl = sparse_ratings(I=7000, J=1070, nnz=1_000_000, B=32, name=name)
    elif name == "paper_poisson_1024":
        # the paper's synthetic Poisson NMF, fully observed.  Its step size
        # (0.01 / t)^0.51 diverges within a few iterations under this
        # gradient scaling (N / |part| times the part's sum), so the step
        # constant comes from the stability rule with the paper's decay
        wl = dense_poisson(I=1024, J=1024, K=32, B=32, heldout=0.0, data_seed=1010, chain_seed=2010,
                           T=10_000, burn_in=5_000, thin=10, name=name)
        wl.eps_a = step_scale(wl.row, wl.col, wl.val, wl.I, wl.J, wl.beta, wl.phi)
        return wl
    elif name == "paper_poisson_512":
        wl = dense_poisson(I=512, J=512, K=32, B=16, heldout=0.0, data_seed=1012, chain_seed=2012,
                           T=10_000, burn_in=5_000, thin=10, name=name)
        wl.eps_a = step_scale(wl.row, wl.col, wl.val, wl.I, wl.J, wl.beta, wl.phi)
        return wl
    elif name == "paper_cpoisson_1024":
        return paper_compound_poisson()
    elif name == "paper_spectrum_256":
        return dense_poisson(I=256, J=256, K=8, B=8, heldout=0.0, data_seed=1011, chain_seed=2011,
                             T=10_000, burn_in=5_000, thin=10, eps_a=1e-3, eps_t0=1.0, eps_gamma=0.51, name=name)
    else:
        raise KeyError(f"unknown workload {name}")
    wl.thin = 10
    return wl

