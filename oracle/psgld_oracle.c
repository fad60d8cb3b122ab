/*
 * psgld_oracle.c -- plain FP64 CPU reference of Parallel SGLD (PSGLD) for
 * matrix factorisation (Simsekli et al., "Parallel Stochastic Gradient Markov
 * Chain Monte Carlo for Matrix Factorisation Models", arXiv:1506.01418).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It is slow on purpose: every step is written in the order
 * the paper gives it, in double precision, with sequential sums.  Nothing in
 * the product path (the HIP library and its Python binding) may link, import
 * or call it; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no source with the GPU library.
 *
 * What it computes (0-based iteration t; the paper counts t = 1..T):
 *   - Model, Section 4 Eq. (13): v_ij ~ TW(mu_ij, phi, beta) with
 *     mu_ij = sum_k w_ik h_kj and log TW = -d_beta(v||mu)/phi + const;
 *     priors exponential (rate lambda, on |x|) or Gaussian (precision lambda).
 *   - Blocks and parts, Section 3 Definitions 1-2: contiguous partitions of
 *     [I] and [J] into B pieces; part p = { (b, (b+p) mod B) : b = 0..B-1 },
 *     chosen in cyclic order p = t mod B (Section 4.2.1).
 *   - Update, Eq. (8)-(9): for every block of the part,
 *       x <- x + eps_t * ( N/|Pi_t| * sum_{(i,j) in block} d/dx log p(v_ij|.)
 *                          + d/dx log p(x) ) + N(0, 2 eps_t)
 *     with both gradients taken at the state of iteration t-1, followed by
 *     the optional mirroring x <- |x| (Algorithm 1, Section 3.2).
 *   - Monte Carlo averages after burn-in (Section 4.2.2): FP64 running sums
 *     of x and x^2 at kept iterations, and held-out predictive sums.
 *
 * Threads (OpenMP): the B blocks of a part share no row and no column
 * (Definition 2), so their gradient sums run on different threads, and the
 * rows of W and columns of H are stepped independently.  Every sum keeps
 * the same terms in the same order whatever the thread count, so results
 * are bitwise independent of it.
 *
 * Readings of points the paper leaves open:
 *   N is the number of observed training entries and |Pi_t| the number of
 *   them inside the part; an empty part has scale 0.  eps_t = a (t0 + t)^-gamma
 *   generalises the paper's (a/t)^b.  For beta < 2 the mean is floored,
 *   mu~ = max(mu, mu_floor), before the residual.  Noise: Philox4x32-10
 *   (Salmon et al., SC'11) keyed by (seed lo, seed hi) with counter
 *   (k/4, row-or-column index, t, stream), then Box-Muller.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EARG (-1)
#define OR_ENOMEM (-3)
#define OR_ENUMERIC (-5)

#define OR_FLAG_NOISE_OFF 1u
#define OR_FLAG_FREEZE_W 2u
#define OR_FLAG_FREEZE_H 4u

#define OR_STREAM_W 0u
#define OR_STREAM_H 1u
#define OR_STREAM_PART 4u

/* Part order: cyclic (p = t mod B, the experiments' practice), or drawn at
 * every iteration with probability |part| / N (Condition 2). */
#define OR_ORDER_CYCLIC 0
#define OR_ORDER_RANDOM 1

#define OR_PRIOR_EXPONENTIAL 0
#define OR_PRIOR_GAUSSIAN 1

typedef struct {
    int64_t I, J;
    int32_t K, B;
    double beta, phi, mu_floor;
    int32_t prior_kind, mirror;
    double lambda_w, lambda_h;
    double eps_a, eps_t0, eps_gamma;
    uint64_t seed;
    int64_t burn_in;
    int32_t thin;
    uint32_t flags;
    int32_t part_order;   /* OR_ORDER_CYCLIC or OR_ORDER_RANDOM */
} oracle_cfg;

typedef struct {
    /* data: training entries (any order, no duplicates) and held-out cells */
    int64_t nnz;
    const int32_t *row, *col;
    const double *val;
    int64_t nho;
    const int32_t *hrow, *hcol;
    /* row_piece[i], col_piece[j]: index of the partition piece holding i, j */
    const int32_t *row_piece, *col_piece;
    /* chain state, in/out.  W is I x K row-major, H is K x J row-major. */
    double *W, *H;
    int64_t t;
    double *sumW, *sumW2, *sumH, *sumH2;
    int64_t n_kept;
    double *ho_sum;
    int64_t *ho_cnt;
} oracle_state;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random        */
/* numbers: as easy as 1, 2, 3").  Each round multiplies words 0 and 2 by     */
/* the two 32-bit Philox multipliers, then mixes the high halves with the    */
/* other two words and the round key; the key is bumped by the two Weyl      */
/* constants (golden ratio and sqrt(3)-1 in 32-bit fixed point) between      */
/* rounds.                                                                  */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL_A = 0xD2511F53u;
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u;
static const uint32_t WEYL_A = 0x9E3779B9u;
static const uint32_t WEYL_B = 0xBB67AE85u;

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
        uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
        uint32_t pa_hi = (uint32_t)(pa >> 32), pa_lo = (uint32_t)pa;
        uint32_t pb_hi = (uint32_t)(pb >> 32), pb_lo = (uint32_t)pb;
        uint32_t y0 = pb_hi ^ x1 ^ k0;
        uint32_t y1 = pb_lo;
        uint32_t y2 = pa_hi ^ x3 ^ k1;
        uint32_t y3 = pa_lo;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += WEYL_A;
        k1 += WEYL_B;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* uint32 -> uniform in (0,1): the top 23 bits r>>9 give (2m+1)/2^24, which is
 * exact in binary32 and binary64 and never 0 or 1. */
static double uniform_open(uint32_t r)
{
    return (2.0 * (double)(r >> 9) + 1.0) * (1.0 / 16777216.0);
}

/* Four standard normals for parameters 4q..4q+3 of row-or-column `index` of
 * factor `stream` at iteration t: Box-Muller on (u0,u1) and on (u2,u3).
 * radius[0], radius[1] receive sqrt(-2 ln u0), sqrt(-2 ln u2). */
static void normals4(uint64_t seed, int64_t t, uint32_t stream, int64_t index, int64_t q,
                     double z[4], double radius[2])
{
    uint32_t ctr[4] = {(uint32_t)q, (uint32_t)index, (uint32_t)t, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    for (int pair = 0; pair < 2; ++pair) {
        double u_a = uniform_open(r[2 * pair]);
        double u_b = uniform_open(r[2 * pair + 1]);
        double rad = sqrt(-2.0 * log(u_a));
        double ang = 2.0 * M_PI * u_b;
        z[2 * pair] = rad * cos(ang);
        z[2 * pair + 1] = rad * sin(ang);
        radius[pair] = rad;
    }
}

/* The K normals (and their Box-Muller radii) of one row of W or column of H. */
void oracle_normals(uint64_t seed, int64_t t, uint32_t stream, int64_t index, int32_t K,
                    double *z, double *radius)
{
    for (int64_t q = 0; 4 * q < K; ++q) {
        double z4[4], r2[2];
        normals4(seed, t, stream, index, q, z4, r2);
        for (int m = 0; m < 4; ++m) {
            int64_t k = 4 * q + m;
            if (k < K) {
                z[k] = z4[m];
                if (radius) radius[k] = r2[m / 2];
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Partition (Section 3, the partition P_B(S)): B contiguous pieces; the     */
/* first (n mod B) pieces hold one extra element.                           */
/* ------------------------------------------------------------------------ */
int oracle_partition(int64_t n, int32_t B, int32_t *piece_of)
{
    if (B < 1 || n < B) return OR_EARG;
    int64_t base = n / B, extra = n % B, pos = 0;
    for (int32_t b = 0; b < B; ++b) {
        int64_t len = base + (b < extra ? 1 : 0);
        for (int64_t m = 0; m < len; ++m) piece_of[pos++] = b;
    }
    return OR_OK;
}

/* Part p holds block (b, (b+p) mod B) for every b, so entry (i,j) belongs to
 * part (col_piece - row_piece) mod B. */
static int32_t part_of_entry(int32_t rb, int32_t cb, int32_t B)
{
    return (int32_t)(((cb - rb) % B + B) % B);
}

/* ------------------------------------------------------------------------ */
/* Model pieces.                                                            */
/* ------------------------------------------------------------------------ */

/* Mean used by the likelihood: floored when beta < 2 (the beta-divergence
 * gradient divides by mu^(2-beta)). */
static double floored_mean(const oracle_cfg *c, double mu)
{
    if (c->beta < 2.0 && mu < c->mu_floor) return c->mu_floor;
    return mu;
}

/* d/dmu log TW(v; mu, phi, beta) = -(1/phi) d/dmu d_beta(v||mu)
 *                                = (v - mu) mu^(beta-2) / phi. */
static double residual(const oracle_cfg *c, double v, double mu_t)
{
    return (v - mu_t) * pow(mu_t, c->beta - 2.0) / c->phi;
}

/* d/dx log p(x): exponential with rate lambda on |x| gives -lambda sign(x),
 * sign(0) = +1; Gaussian with precision lambda gives -lambda x. */
static double prior_grad(const oracle_cfg *c, double x, double lambda)
{
    if (c->prior_kind == OR_PRIOR_EXPONENTIAL) return x >= 0.0 ? -lambda : lambda;
    return -lambda * x;
}

/* The likelihood sees |x| when mirroring is on (Section 3.2); d|x|/dx = sign. */
static double model_value(const oracle_cfg *c, double x) { return c->mirror ? fabs(x) : x; }
static double model_sign(const oracle_cfg *c, double x) { return (c->mirror && x < 0.0) ? -1.0 : 1.0; }

/* beta-divergence d_beta(v||mu) (Section 4), with the standard limits at
 * beta = 1 (generalised KL) and beta = 0 (Itakura-Saito). */
double oracle_dbeta(double v, double mu, double beta)
{
    if (beta == 1.0) return (v > 0.0 ? v * log(v / mu) : 0.0) - v + mu;
    if (beta == 0.0) return v / mu - log(v / mu) - 1.0;
    return pow(v, beta) / (beta * (beta - 1.0)) - v * pow(mu, beta - 1.0) / (beta - 1.0) +
           pow(mu, beta) / beta;
}

double oracle_eps(const oracle_cfg *c, int64_t t)
{
    return c->eps_a * pow(c->eps_t0 + (double)t, -c->eps_gamma);
}

/* ------------------------------------------------------------------------ */
/* Entry bookkeeping.  Training entries are put in (i, j) lexicographic      */
/* order (two stable counting sorts: by column, then by row), then bucketed  */
/* stably by (part p, block b) where block b of part p is (b, (b+p) mod B):  */
/* every bucket lists one block's entries in (i, j) order.  Held-out cells   */
/* are bucketed the same way.  The bucketing depends only on the data and   */
/* the pieces, so a chain prepares it once (oracle_prepare).                 */
/* ------------------------------------------------------------------------ */
/* Loops with less work than this many elements run on the calling thread
 * (forking threads costs more than they save on small problems). */
#define OR_PAR_MIN 32768

struct oracle_prep {
    int32_t B;
    int64_t *order;     /* entry ids, bucket-major, (i, j) order inside */
    int64_t *beg;       /* B*B+1 offsets: bucket p*B + b */
    int64_t *ho_order;  /* held-out ids, same bucketing */
    int64_t *ho_beg;
    int64_t *n_part;    /* |Pi_p| for every part */
};
typedef struct oracle_prep oracle_prep;

/* Part p holds block (b, (b+p) mod B) for every b, so entry (i,j) belongs to
 * part (col_piece - row_piece) mod B and, inside it, to block b = row_piece. */
static int64_t bucket_of(const int32_t *rp, const int32_t *cp, int32_t B, int32_t i, int32_t j)
{
    return (int64_t)part_of_entry(rp[i], cp[j], B) * B + rp[i];
}

/* Stable counting sort of the ids in[0..n) by key[id] in [0, nkey). */
static int counting_sort(const int64_t *in, int64_t n, const int32_t *key, int64_t nkey, int64_t *out)
{
    int64_t *cnt = (int64_t *)calloc((size_t)nkey + 1, sizeof(int64_t));
    if (!cnt) return OR_ENOMEM;
    for (int64_t m = 0; m < n; ++m) cnt[key[in[m]] + 1]++;
    for (int64_t k = 0; k < nkey; ++k) cnt[k + 1] += cnt[k];
    for (int64_t m = 0; m < n; ++m) out[cnt[key[in[m]]]++] = in[m];
    free(cnt);
    return OR_OK;
}

static int bucket_entries(const oracle_cfg *c, const int32_t *rp, const int32_t *cp, int64_t n,
                          const int32_t *row, const int32_t *col, int64_t **order_out, int64_t **beg_out)
{
    int32_t B = c->B;
    int64_t nb = (int64_t)B * B;
    int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *beg = (int64_t *)calloc((size_t)nb + 1, sizeof(int64_t));
    int rc = (ids && tmp && order && beg) ? OR_OK : OR_ENOMEM;
    if (rc == OR_OK) {
        for (int64_t e = 0; e < n; ++e) ids[e] = e;
        rc = counting_sort(ids, n, col, c->J, tmp);            /* by column ... */
        if (rc == OR_OK) rc = counting_sort(tmp, n, row, c->I, ids);   /* ... then by row: (i, j) order */
    }
    if (rc == OR_OK) {
        for (int64_t m = 0; m < n; ++m) beg[bucket_of(rp, cp, B, row[ids[m]], col[ids[m]]) + 1]++;
        for (int64_t k = 0; k < nb; ++k) beg[k + 1] += beg[k];
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
        if (!fill) {
            rc = OR_ENOMEM;
        } else {
            memcpy(fill, beg, sizeof(int64_t) * (size_t)nb);
            for (int64_t m = 0; m < n; ++m) order[fill[bucket_of(rp, cp, B, row[ids[m]], col[ids[m]])]++] = ids[m];
            free(fill);
        }
    }
    free(ids);
    free(tmp);
    if (rc != OR_OK) {
        free(order);
        free(beg);
        return rc;
    }
    *order_out = order;
    *beg_out = beg;
    return OR_OK;
}

static int check_inputs(const oracle_cfg *c, const oracle_state *s)
{
    if (c->I < 1 || c->J < 1 || c->K < 1 || c->B < 1 || c->B > c->I || c->B > c->J) return OR_EARG;
    if (!(c->phi > 0.0) || !(c->lambda_w > 0.0) || !(c->lambda_h > 0.0)) return OR_EARG;
    for (int64_t e = 0; e < s->nnz; ++e) {
        if (s->row[e] < 0 || s->row[e] >= c->I || s->col[e] < 0 || s->col[e] >= c->J) return OR_EARG;
    }
    for (int64_t e = 0; e < s->nho; ++e) {
        if (s->hrow[e] < 0 || s->hrow[e] >= c->I || s->hcol[e] < 0 || s->hcol[e] >= c->J) return OR_EARG;
    }
    return OR_OK;
}

void oracle_release(oracle_prep *pr)
{
    if (!pr) return;
    free(pr->order);
    free(pr->beg);
    free(pr->ho_order);
    free(pr->ho_beg);
    free(pr->n_part);
    free(pr);
}

/* Buckets the training entries and held-out cells of s under c's pieces.
 * Returns NULL on invalid input or when memory runs out. */
oracle_prep *oracle_prepare(const oracle_cfg *c, const oracle_state *s)
{
    if (check_inputs(c, s)) return NULL;
    oracle_prep *pr = (oracle_prep *)calloc(1, sizeof(oracle_prep));
    if (!pr) return NULL;
    pr->B = c->B;
    pr->n_part = (int64_t *)calloc((size_t)c->B, sizeof(int64_t));
    if (!pr->n_part ||
        bucket_entries(c, s->row_piece, s->col_piece, s->nnz, s->row, s->col, &pr->order, &pr->beg) ||
        bucket_entries(c, s->row_piece, s->col_piece, s->nho, s->hrow, s->hcol, &pr->ho_order, &pr->ho_beg)) {
        oracle_release(pr);
        return NULL;
    }
    for (int32_t p = 0; p < c->B; ++p)
        pr->n_part[p] = pr->beg[(int64_t)(p + 1) * c->B] - pr->beg[(int64_t)p * c->B];
    return pr;
}

/* Threads used by the parallel loops (OpenMP); n < 1 leaves the setting. */
int oracle_threads(int n)
{
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* Number of training entries in each part, |Pi_p|. */
int oracle_part_sizes(const oracle_cfg *c, const oracle_state *s, int64_t *n_p)
{
    for (int32_t p = 0; p < c->B; ++p) n_p[p] = 0;
    for (int64_t e = 0; e < s->nnz; ++e)
        n_p[part_of_entry(s->row_piece[s->row[e]], s->col_piece[s->col[e]], c->B)]++;
    return OR_OK;
}

/* Likelihood gradient of one part, scaled by N/|Pi_p|, at the state in s.
 * gW (I x K) and gH (K x J) are overwritten.  When gpW/gpH are non-NULL they
 * receive the matching absolute-value bound
 *   sum_j (|v| + sum_k' |w_ik' h_k'j|) mu~^(beta-2)/phi |h_kj|   (times the scale),
 * used to scale the rounding tolerance of a single GPU step.
 * The blocks of the part share no row and no column (Definition 2), so they
 * are summed independently (one thread per block at a time); inside a block
 * the entries are visited in (i,j) lexicographic order with sequential sums,
 * so every sum has the same terms in the same order for any thread count. */
static void part_gradient(const oracle_cfg *c, const oracle_state *s, const oracle_prep *pr, int32_t p,
                          double scale, double *gW, double *gH, double *gpW, double *gpH)
{
    int64_t I = c->I, J = c->J;
    int32_t K = c->K, B = c->B;
#pragma omp parallel for schedule(static) if (I * K >= OR_PAR_MIN)
    for (int64_t m = 0; m < I * K; ++m) {
        gW[m] = 0.0;
        if (gpW) gpW[m] = 0.0;
    }
#pragma omp parallel for schedule(static) if ((int64_t)K * J >= OR_PAR_MIN)
    for (int64_t m = 0; m < (int64_t)K * J; ++m) {
        gH[m] = 0.0;
        if (gpH) gpH[m] = 0.0;
    }
    const int64_t part_work = (pr->beg[(int64_t)(p + 1) * B] - pr->beg[(int64_t)p * B]) * K;
#pragma omp parallel for schedule(dynamic, 1) if (part_work >= OR_PAR_MIN)
    for (int32_t b = 0; b < B; ++b) {
        int64_t beg = pr->beg[(int64_t)p * B + b], end = pr->beg[(int64_t)p * B + b + 1];
        for (int64_t n = beg; n < end; ++n) {
            int64_t e = pr->order[n];
            int64_t i = s->row[e], j = s->col[e];
            double v = s->val[e];
            double mu = 0.0, mu_abs = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                double prod = model_value(c, s->W[i * K + k]) * model_value(c, s->H[k * J + j]);
                mu += prod;
                mu_abs += fabs(prod);
            }
            double mu_t = floored_mean(c, mu);
            double e_ij = residual(c, v, mu_t);
            double e_abs = (fabs(v) + mu_abs) * pow(mu_t, c->beta - 2.0) / c->phi;
            for (int32_t k = 0; k < K; ++k) {
                double w = s->W[i * K + k], h = s->H[k * J + j];
                gW[i * K + k] += e_ij * model_value(c, h) * model_sign(c, w);
                gH[k * J + j] += e_ij * model_value(c, w) * model_sign(c, h);
                if (gpW) gpW[i * K + k] += e_abs * fabs(h);
                if (gpH) gpH[k * J + j] += e_abs * fabs(w);
            }
        }
    }
#pragma omp parallel for schedule(static) if (I * K >= OR_PAR_MIN)
    for (int64_t m = 0; m < I * K; ++m) {
        gW[m] *= scale;
        if (gpW) gpW[m] *= scale;
    }
#pragma omp parallel for schedule(static) if ((int64_t)K * J >= OR_PAR_MIN)
    for (int64_t m = 0; m < (int64_t)K * J; ++m) {
        gH[m] *= scale;
        if (gpH) gpH[m] *= scale;
    }
}

static double part_scale(int64_t N, int64_t n_p)
{
    return n_p > 0 ? (double)N / (double)n_p : 0.0;
}

/* Drift of the part-estimated log joint, Section 3.1:
 *   d/dtheta L^_p(theta) = N/|Pi_p| sum_{Pi_p} d/dtheta log p(v|theta) + d/dtheta log p(theta),
 * at the state in s.  dW is I x K, dH is K x J. */
int oracle_drift(const oracle_cfg *c, const oracle_state *s, int32_t p, double *dW, double *dH)
{
    int rc = check_inputs(c, s);
    if (rc) return rc;
    if (p < 0 || p >= c->B) return OR_EARG;
    oracle_prep *pr = oracle_prepare(c, s);
    if (!pr) return OR_ENOMEM;
    double scale = part_scale(s->nnz, pr->n_part[p]);
    part_gradient(c, s, pr, p, scale, dW, dH, NULL, NULL);
    for (int64_t m = 0; m < c->I * c->K; ++m) dW[m] += prior_grad(c, s->W[m], c->lambda_w);
    for (int64_t m = 0; m < (int64_t)c->K * c->J; ++m) dH[m] += prior_grad(c, s->H[m], c->lambda_h);
    oracle_release(pr);
    return OR_OK;
}

/* Training log-likelihood -sum d_beta(v||mu~)/phi (the normaliser of the
 * Tweedie density does not depend on W, H and is dropped, Section 4). */
int oracle_loglik(const oracle_cfg *c, const oracle_state *s, double *ll)
{
    int rc = check_inputs(c, s);
    if (rc) return rc;
    int64_t J = c->J;
    int32_t K = c->K;
    double acc = 0.0;
    for (int64_t e = 0; e < s->nnz; ++e) {
        int64_t i = s->row[e], j = s->col[e];
        double mu = 0.0;
        for (int32_t k = 0; k < K; ++k)
            mu += model_value(c, s->W[i * K + k]) * model_value(c, s->H[k * J + j]);
        acc -= oracle_dbeta(s->val[e], floored_mean(c, mu), c->beta) / c->phi;
    }
    *ll = acc;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1.  Runs n_iter iterations from s->t.  If bound_W / bound_H are */
/* non-NULL they receive, for the last iteration run, the per-parameter      */
/* magnitude scale                                                          */
/*   c_x = |x_old| + eps (s_p G+_x + |prior'(x_old)|) + sigma R_x            */
/* (R_x: Box-Muller radius of x's normal) that GPU rounding is measured in.  */
/* ------------------------------------------------------------------------ */
/* Part of iteration t.  Random order (Condition 2): one Philox block with
 * counter (0, 0, t, PART stream) gives u = (2 (r0 >> 9) + 1) 2^-24 in (0,1);
 * the part is the first p with u N < n_0 + ... + n_p, so part p is drawn
 * with probability n_p / N (up to the 2^-23 resolution of u) and a part
 * without entries never.  The comparison is made on integers scaled by 2^24,
 * exactly.  Without any entry (N = 0) the order is cyclic. */
int32_t oracle_part_at(const oracle_cfg *c, int64_t t, const int64_t *n_p, int64_t N)
{
    if (c->part_order != OR_ORDER_RANDOM || N <= 0) return (int32_t)(t % c->B);
    const uint32_t ctr[4] = {0u, 0u, (uint32_t)t, OR_STREAM_PART};
    const uint32_t key[2] = {(uint32_t)c->seed, (uint32_t)(c->seed >> 32)};
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    const uint64_t scaled_u = 2ull * (uint64_t)(r[0] >> 9) + 1ull;   /* u * 2^24 */
    const uint64_t lhs = scaled_u * (uint64_t)N;
    uint64_t cum = 0;
    for (int32_t p = 0; p < c->B; ++p) {
        cum += (uint64_t)n_p[p];
        if (lhs < (cum << 24)) return p;
    }
    return c->B - 1;
}

/* Langevin step of one factor row (W, stride 1 over k) or column (H, stride
 * J over k): x <- x + eps (g + prior'(x)) + sigma z, then |x| if mirroring,
 * with z the K normals of that row or column at iteration t.  z and rad are
 * K-long work arrays of the calling thread. */
static void step_vector(const oracle_cfg *c, int64_t t, uint32_t stream, int64_t index, double lambda,
                        double eps, double sigma, double *x, int64_t stride, const double *g, const double *gp,
                        double *bound, double *z, double *rad)
{
    int32_t K = c->K;
    if (c->flags & OR_FLAG_NOISE_OFF) {
        for (int32_t k = 0; k < K; ++k) { z[k] = 0.0; rad[k] = 0.0; }
    } else {
        oracle_normals(c->seed, t, stream, index, K, z, rad);
    }
    for (int32_t k = 0; k < K; ++k) {
        int64_t m = k * stride;
        double xo = x[m];
        double pg = prior_grad(c, xo, lambda);
        double xn = xo + eps * (g[m] + pg) + sigma * z[k];
        if (c->mirror) xn = fabs(xn);
        if (bound) bound[m] = fabs(xo) + eps * (gp[m] + fabs(pg)) + sigma * rad[k];
        x[m] = xn;
    }
}

int oracle_run_prepared(const oracle_cfg *c, oracle_state *s, const oracle_prep *pr, int64_t n_iter,
                        double *bound_W, double *bound_H)
{
    int rc = check_inputs(c, s);
    if (rc) return rc;
    if (c->thin < 1 || !pr || pr->B != c->B) return OR_EARG;
    int64_t I = c->I, J = c->J;
    int32_t K = c->K, B = c->B;

    double *gW = (double *)malloc(sizeof(double) * (size_t)(I * K));
    double *gH = (double *)malloc(sizeof(double) * (size_t)(K * J));
    double *gpW = bound_W ? (double *)malloc(sizeof(double) * (size_t)(I * K)) : NULL;
    double *gpH = bound_H ? (double *)malloc(sizeof(double) * (size_t)(K * J)) : NULL;
    if (!gW || !gH || (bound_W && !gpW) || (bound_H && !gpH)) {
        rc = OR_ENOMEM;
        goto done;
    }

    for (int64_t it = 0; it < n_iter; ++it) {
        int64_t t = s->t;
        /* Set the step size; pick the part. */
        double eps = oracle_eps(c, t);
        double sigma = sqrt(2.0 * eps);
        int32_t p = oracle_part_at(c, t, pr->n_part, s->nnz);
        double scale = part_scale(s->nnz, pr->n_part[p]);
        int last = (it == n_iter - 1);

        /* Held-out predictive sums use the state before this update; every
         * cell has its own sum. */
        if (t >= c->burn_in) {
            int64_t h0 = pr->ho_beg[(int64_t)p * B], h1 = pr->ho_beg[(int64_t)(p + 1) * B];
#pragma omp parallel for schedule(static) if ((h1 - h0) * K >= OR_PAR_MIN)
            for (int64_t n = h0; n < h1; ++n) {
                int64_t e = pr->ho_order[n];
                int64_t i = s->hrow[e], j = s->hcol[e];
                double mu = 0.0;
                for (int32_t k = 0; k < K; ++k)
                    mu += model_value(c, s->W[i * K + k]) * model_value(c, s->H[k * J + j]);
                s->ho_sum[e] += mu;
                s->ho_cnt[e] += 1;
            }
        }

        /* Likelihood gradient over the part, at the old state (Eq. 8-9). */
        part_gradient(c, s, pr, p, scale, gW, gH, last ? gpW : NULL, last ? gpH : NULL);

        /* Every row of W and every column of H lies in exactly one block of
         * the part (Definition 2), so the update sweeps all of W and H; each
         * row and column is stepped independently. */
        if (!(c->flags & OR_FLAG_FREEZE_W)) {
#pragma omp parallel if (I * K >= OR_PAR_MIN / 8)
            {
                double *z = (double *)malloc(sizeof(double) * (size_t)K);
                double *rad = (double *)malloc(sizeof(double) * (size_t)K);
#pragma omp for schedule(static)
                for (int64_t i = 0; i < I; ++i)
                    if (z && rad)
                        step_vector(c, t, OR_STREAM_W, i, c->lambda_w, eps, sigma, s->W + i * K, 1, gW + i * K,
                                    (last && bound_W) ? gpW + i * K : NULL, (last && bound_W) ? bound_W + i * K : NULL,
                                    z, rad);
                if (!z || !rad) {
#pragma omp atomic write
                    rc = OR_ENOMEM;
                }
                free(z);
                free(rad);
            }
            if (rc) goto done;
        } else if (last && bound_W) {
            for (int64_t m = 0; m < I * K; ++m) bound_W[m] = fabs(s->W[m]);
        }
        if (!(c->flags & OR_FLAG_FREEZE_H)) {
#pragma omp parallel if ((int64_t)K * J >= OR_PAR_MIN / 8)
            {
                double *z = (double *)malloc(sizeof(double) * (size_t)K);
                double *rad = (double *)malloc(sizeof(double) * (size_t)K);
#pragma omp for schedule(static)
                for (int64_t j = 0; j < J; ++j)
                    if (z && rad)
                        step_vector(c, t, OR_STREAM_H, j, c->lambda_h, eps, sigma, s->H + j, J, gH + j,
                                    (last && bound_H) ? gpH + j : NULL, (last && bound_H) ? bound_H + j : NULL,
                                    z, rad);
                if (!z || !rad) {
#pragma omp atomic write
                    rc = OR_ENOMEM;
                }
                free(z);
                free(rad);
            }
            if (rc) goto done;
        } else if (last && bound_H) {
            for (int64_t m = 0; m < (int64_t)K * J; ++m) bound_H[m] = fabs(s->H[m]);
        }

        /* Monte Carlo sums of the new sample at kept iterations. */
        if (t >= c->burn_in && (t - c->burn_in) % c->thin == 0) {
#pragma omp parallel for schedule(static) if (I * K >= OR_PAR_MIN)
            for (int64_t m = 0; m < I * K; ++m) {
                s->sumW[m] += s->W[m];
                s->sumW2[m] += s->W[m] * s->W[m];
            }
#pragma omp parallel for schedule(static) if ((int64_t)K * J >= OR_PAR_MIN)
            for (int64_t m = 0; m < (int64_t)K * J; ++m) {
                s->sumH[m] += s->H[m];
                s->sumH2[m] += s->H[m] * s->H[m];
            }
            s->n_kept += 1;
        }
        s->t = t + 1;

        int bad = 0;
#pragma omp parallel for schedule(static) reduction(|| : bad) if (I * K >= OR_PAR_MIN)
        for (int64_t m = 0; m < I * K; ++m) bad = bad || !isfinite(s->W[m]);
#pragma omp parallel for schedule(static) reduction(|| : bad) if ((int64_t)K * J >= OR_PAR_MIN)
        for (int64_t m = 0; m < (int64_t)K * J; ++m) bad = bad || !isfinite(s->H[m]);
        if (bad) { rc = OR_ENUMERIC; goto done; }
    }

done:
    free(gW); free(gH); free(gpW); free(gpH);
    return rc;
}

/* One-shot form: buckets the data, runs, and frees the buckets. */
int oracle_run(const oracle_cfg *c, oracle_state *s, int64_t n_iter, double *bound_W, double *bound_H)
{
    int rc = check_inputs(c, s);
    if (rc) return rc;
    oracle_prep *pr = oracle_prepare(c, s);
    if (!pr) return OR_ENOMEM;
    rc = oracle_run_prepared(c, s, pr, n_iter, bound_W, bound_H);
    oracle_release(pr);
    return rc;
}
