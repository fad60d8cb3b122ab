/* A plain C user of the library's ABI (include/psgld.h), for the tests: no
 * Python and no PyTorch in the process.
 *
 * usage: c_abi_driver <dir> <n_iter>
 * <dir>/problem.txt  : I J K B beta phi prior(0 exp, 1 gauss) lambda_w lambda_h mirror seed
 *                      eps_a eps_t0 eps_gamma nnz  (whitespace separated)
 * <dir>/row.i32, col.i32, val.f32, W0.f32 (I x K), H0.f32 (K x J): raw arrays
 * Runs psgld_step(n_iter) from t = 0 on the library's own stream and device
 * memory, then writes <dir>/W.f32 and <dir>/H.f32 (the current sample) and
 * <dir>/mean_W.f64, <dir>/mean_H.f64 when n_iter passes burn-in 0 (moments
 * are kept from t = 0 here).  Exit status 0 on success, else prints the
 * library's error message. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "psgld.h"

static void *read_file(const char *dir, const char *name, size_t bytes)
{
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        exit(2);
    }
    void *p = malloc(bytes ? bytes : 1);
    if (fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read on %s\n", path);
        exit(2);
    }
    fclose(f);
    return p;
}

static void write_file(const char *dir, const char *name, const void *p, size_t bytes)
{
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot write %s\n", path);
        exit(2);
    }
    fclose(f);
}

#define CHECK(call)                                                                \
    do {                                                                           \
        psgld_status st_ = (call);                                                 \
        if (st_ != PSGLD_OK) {                                                     \
            fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_,               \
                    psgld_last_error(ctx));                                        \
            return 1;                                                              \
        }                                                                          \
    } while (0)

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s <dir> <n_iter>\n", argv[0]);
        return 2;
    }
    const char *dir = argv[1];
    const long long n_iter = atoll(argv[2]);
    char path[4096];
    snprintf(path, sizeof path, "%s/problem.txt", dir);
    FILE *f = fopen(path, "r");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        return 2;
    }
    long long I, J, nnz, seed;
    int K, B, prior_kind, mirror;
    double beta, phi, lw, lh, ea, et0, eg;
    if (fscanf(f, "%lld %lld %d %d %lf %lf %d %lf %lf %d %lld %lf %lf %lf %lld", &I, &J, &K, &B, &beta, &phi,
               &prior_kind, &lw, &lh, &mirror, &seed, &ea, &et0, &eg, &nnz) != 15) {
        fprintf(stderr, "bad problem file\n");
        return 2;
    }
    fclose(f);
    int32_t *row = read_file(dir, "row.i32", (size_t)nnz * 4);
    int32_t *col = read_file(dir, "col.i32", (size_t)nnz * 4);
    float *val = read_file(dir, "val.f32", (size_t)nnz * 4);
    float *W0 = read_file(dir, "W0.f32", (size_t)I * K * 4);
    float *H0 = read_file(dir, "H0.f32", (size_t)K * J * 4);

    psgld_likelihood lik = {beta, phi};
    psgld_prior prior = {prior_kind, lw, lh, mirror};
    psgld_options opt;
    psgld_default_options(&opt);
    opt.seed = (uint64_t)seed;
    opt.burn_in = 0;
    opt.thin = 1;
    psgld_ctx *ctx = NULL;
    psgld_status st = psgld_create(I, J, K, B, &lik, &prior, &opt, &ctx);
    if (st != PSGLD_OK) {
        fprintf(stderr, "psgld_create failed (%d): %s\n", (int)st, psgld_last_error(NULL));
        return 1;
    }
    CHECK(psgld_load_coo(ctx, nnz, row, col, val));
    CHECK(psgld_set_factors(ctx, W0, H0));
    psgld_eps_schedule sched = {ea, et0, eg};
    CHECK(psgld_step(ctx, n_iter, &sched));
    CHECK(psgld_sync(ctx));
    float *W = malloc((size_t)I * K * 4), *H = malloc((size_t)K * J * 4);
    CHECK(psgld_get_factors(ctx, W, H));
    write_file(dir, "W.f32", W, (size_t)I * K * 4);
    write_file(dir, "H.f32", H, (size_t)K * J * 4);
    if (n_iter > 0) {
        double *mW = malloc((size_t)I * K * 8), *mH = malloc((size_t)K * J * 8);
        CHECK(psgld_posterior_mean(ctx, mW, mH));
        write_file(dir, "mean_W.f64", mW, (size_t)I * K * 8);
        write_file(dir, "mean_H.f64", mH, (size_t)K * J * 8);
        free(mW);
        free(mH);
    }
    psgld_destroy(ctx);
    printf("c_abi_driver: %lld iterations of %lld x %lld, K = %d, B = %d\n", n_iter, I, J, K, B);
    free(W);
    free(H);
    free(row);
    free(col);
    free(val);
    free(W0);
    free(H0);
    return 0;
}
