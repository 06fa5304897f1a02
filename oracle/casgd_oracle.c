/*
 * FP64 CPU oracle for s-step (communication-avoiding) mini-batch SGD on
 * L2-regularised logistic regression.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library, its kernels or its
 * Python binding may include, link or call this file. Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark use it. It shares no
 * code, header, table or constant generator with the GPU path.
 *
 * Everything is computed in IEEE double, in plain loops, in the order the
 * definitions are written. Data enters as FP64 (callers pass the exact FP64
 * value of whatever storage format the GPU uses), and every inner product
 * is a left-to-right sum.
 *
 * Definitions followed (paper = "Mixed-Precision Communication-Avoiding SGD
 * for Generalized Linear Models on GPUs"):
 *  - empirical risk and the three losses of Sec. 2.1: logistic
 *    L(r,y) = log(1+exp(-y r)), linear L = (r-y)^2/2, Poisson L = exp(r) - y r;
 *  - residuals delta = -dL/dr (Sec. 3.1): y (1 - sigma(y r)), y - r and
 *    y - exp(r);
 *  - mini-batch SGD step in delta form x <- x + (eta/b) Y^T delta: Sec. 3.1
 *    and Sec. 2.1; with the L2 term (lambda/2)||x||^2 (not in the paper) the
 *    step becomes x <- (1 - eta*lambda) x + (eta/b) Y^T delta;
 *  - the s-step outer iteration: Algorithm 1 (sample sb rows, r = Y x,
 *    G = Y Y^T, s residual corrections on the strict block-lower part of G,
 *    then one update with Y^T delta_hist). With the decay beta = 1 - eta*lambda
 *    the corrected margin of inner step j is
 *        z_j = beta^j r_j + (eta/b) sum_{i<j} beta^(j-1-i) G_{j,i} delta_i
 *    and the update is x <- beta^s x + (eta/b) Y^T c, c_i = beta^(s-1-i) delta_i;
 *    for lambda = 0 this is Algorithm 1 unchanged.
 *  - sampling: s*b indices i.i.d. uniform with replacement (Algorithm 1,
 *    first step). The paper does not fix the generator; this oracle uses
 *    SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) as a counter-based
 *    stream: sample number t of seed k is mix(k + (t+1)*gamma), mapped to
 *    [0, m) by the high 64 bits of the 128-bit product with m. Block j of
 *    outer iteration h holds samples h*s*b + j*b ... h*s*b + (j+1)*b - 1, so
 *    plain SGD step k (samples k*b ...) sees exactly the same rows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OMP_MIN_WORK 65536

/* ---------------------------------------------------------------- sampling */

static uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t oracle_splitmix64(uint64_t seed, uint64_t t)
{
    return sm64_mix(seed + (t + 1) * 0x9e3779b97f4a7c15ULL);
}

int64_t oracle_sample_index(uint64_t seed, uint64_t t, int64_t m)
{
    unsigned __int128 p = (unsigned __int128)oracle_splitmix64(seed, t) * (uint64_t)m;
    return (int64_t)(p >> 64);
}

void oracle_sample_indices(uint64_t seed, uint64_t t0, int64_t count, int64_t m,
                           int64_t *out)
{
    for (int64_t q = 0; q < count; ++q)
        out[q] = oracle_sample_index(seed, t0 + (uint64_t)q, m);
}

/* ------------------------------------------------------------- loss pieces */

/* Loss selector: 0 logistic, 1 linear (least squares), 2 Poisson (Sec. 2.1). */
enum { LOSS_LOGISTIC = 0, LOSS_LINEAR = 1, LOSS_POISSON = 2 };

/* delta(z, y) = -dL/dz (Sec. 3.1). Logistic: y / (1 + exp(y z)), which equals
 * y (1 - sigma(y z)); linear: y - z; Poisson: y - exp(z). */
static double glm_delta(double z, double y, int loss)
{
    if (loss == LOSS_LINEAR)
        return y - z;
    if (loss == LOSS_POISSON)
        return y - exp(z);
    return y / (1.0 + exp(y * z));
}

static double logistic_delta(double z, double y) { return glm_delta(z, y, LOSS_LOGISTIC); }

double oracle_delta(double z, double y) { return logistic_delta(z, y); }
double oracle_delta_glm(double z, double y, int32_t loss) { return glm_delta(z, y, loss); }

/* softplus(v) = log(1 + exp(v)), evaluated without overflow. */
static double softplus(double v)
{
    return (v > 0 ? v : 0.0) + log1p(exp(-fabs(v)));
}

/* L(z, y) of Sec. 2.1; the logistic form through the stable softplus. */
static double glm_loss(double z, double y, int loss)
{
    if (loss == LOSS_LINEAR)
        return 0.5 * (z - y) * (z - y);
    if (loss == LOSS_POISSON)
        return exp(z) - y * z;
    return softplus(-y * z);
}

/* Mean loss m^-1 sum L(a_i^T x, y_i) over dense rows. */
static double mean_loss_f64(const double *X, int64_t ld, int64_t m, int64_t n,
                            const double *y, const double *x, int loss)
{
    double total = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        const double *a = X + i * ld;
        double z = 0.0;
        for (int64_t k = 0; k < n; ++k)
            z += a[k] * x[k];
        total += glm_loss(z, y[i], loss);
    }
    return m > 0 ? total / (double)m : 0.0;
}

static double mean_loss_f32(const float *X, int64_t ld, int64_t m, int64_t n,
                            const float *y, const double *x, int loss)
{
    double total = 0.0;
#pragma omp parallel for reduction(+ : total) schedule(static) if (m * n > OMP_MIN_WORK)
    for (int64_t i = 0; i < m; ++i) {
        const float *a = X + i * ld;
        double z = 0.0;
        for (int64_t k = 0; k < n; ++k)
            z += (double)a[k] * x[k];
        total += glm_loss(z, (double)y[i], loss);
    }
    return m > 0 ? total / (double)m : 0.0;
}

static double mean_loss_csr(const int64_t *row_ptr, const int32_t *col_idx,
                            const double *val, int64_t m, const double *y,
                            const double *x, int loss)
{
    double total = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double z = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            z += val[p] * x[col_idx[p]];
        total += glm_loss(z, y[i], loss);
    }
    return m > 0 ? total / (double)m : 0.0;
}

/* Mean logistic loss m^-1 sum log(1 + exp(-y_i a_i^T x)) over dense rows. */
double oracle_logloss(const double *X, int64_t ld, int64_t m, int64_t n,
                      const double *y, const double *x)
{
    return mean_loss_f64(X, ld, m, n, y, x, LOSS_LOGISTIC);
}

double oracle_logloss_f32(const float *X, int64_t ld, int64_t m, int64_t n,
                          const float *y, const double *x)
{
    return mean_loss_f32(X, ld, m, n, y, x, LOSS_LOGISTIC);
}

double oracle_logloss_csr(const int64_t *row_ptr, const int32_t *col_idx,
                          const double *val, int64_t m, const double *y,
                          const double *x)
{
    return mean_loss_csr(row_ptr, col_idx, val, m, y, x, LOSS_LOGISTIC);
}

double oracle_loss_glm(const double *X, int64_t ld, int64_t m, int64_t n,
                       const double *y, const double *x, int32_t loss)
{
    return mean_loss_f64(X, ld, m, n, y, x, loss);
}

double oracle_loss_glm_f32(const float *X, int64_t ld, int64_t m, int64_t n,
                           const float *y, const double *x, int32_t loss)
{
    return mean_loss_f32(X, ld, m, n, y, x, loss);
}

double oracle_loss_glm_csr(const int64_t *row_ptr, const int32_t *col_idx,
                           const double *val, int64_t m, const double *y,
                           const double *x, int32_t loss)
{
    return mean_loss_csr(row_ptr, col_idx, val, m, y, x, loss);
}

/* ------------------------------------------------------------- dense rows */

/* Element accessor for the two input storage types the oracle accepts. The
 * float path exists so that large FP32 matrices need not be copied to FP64;
 * every element is promoted exactly. */
typedef struct {
    const void *p;
    int is_f32;
    int64_t ld;
} rows_t;

static void gather_rows(rows_t X, int64_t n, const int64_t *idx, int64_t cnt,
                        double *Y)
{
    for (int64_t q = 0; q < cnt; ++q) {
        if (X.is_f32) {
            const float *a = (const float *)X.p + idx[q] * X.ld;
            for (int64_t k = 0; k < n; ++k)
                Y[q * n + k] = (double)a[k];
        } else {
            const double *a = (const double *)X.p + idx[q] * X.ld;
            memcpy(Y + q * n, a, (size_t)n * sizeof(double));
        }
    }
}

/* z_q = Y_q . x for q < cnt */
static void rows_times_x(const double *Y, int64_t cnt, int64_t n, const double *x,
                         double *z)
{
#pragma omp parallel for schedule(static) if (cnt * n > OMP_MIN_WORK)
    for (int64_t q = 0; q < cnt; ++q) {
        double acc = 0.0;
        for (int64_t k = 0; k < n; ++k)
            acc += Y[q * n + k] * x[k];
        z[q] = acc;
    }
}

/* x_k <- decay * x_k + alpha * sum_q Y_qk w_q (sum over q in order) */
static void decay_plus_yt_w(const double *Y, int64_t cnt, int64_t n,
                            const double *w, double decay, double alpha, double *x)
{
#pragma omp parallel for schedule(static) if (cnt * n > OMP_MIN_WORK)
    for (int64_t k = 0; k < n; ++k) {
        double acc = 0.0;
        for (int64_t q = 0; q < cnt; ++q)
            acc += Y[q * n + k] * w[q];
        x[k] = decay * x[k] + alpha * acc;
    }
}

/* Plain mini-batch SGD (steps step0 .. step0+nsteps-1), in place on x. */
static int sgd_impl(rows_t X, int64_t m, int64_t n, const double *y,
                    const float *y32, double *x, double eta, double lambda,
                    int32_t b, uint64_t seed, uint64_t step0, int64_t nsteps, int loss)
{
    if (m <= 0 || n <= 0 || b <= 0)
        return -1;
    const double alpha = eta / (double)b;
    const double beta = 1.0 - eta * lambda;
    double *Y = (double *)malloc(sizeof(double) * (size_t)b * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)b);
    double *d = (double *)malloc(sizeof(double) * (size_t)b);
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)b);
    if (!Y || !z || !d || !idx) {
        free(Y); free(z); free(d); free(idx);
        return -3;
    }
    for (int64_t st = 0; st < nsteps; ++st) {
        uint64_t k = step0 + (uint64_t)st;
        oracle_sample_indices(seed, k * (uint64_t)b, b, m, idx);
        gather_rows(X, n, idx, b, Y);
        rows_times_x(Y, b, n, x, z);
        for (int32_t q = 0; q < b; ++q) {
            double yq = y ? y[idx[q]] : (double)y32[idx[q]];
            d[q] = glm_delta(z[q], yq, loss);
        }
        decay_plus_yt_w(Y, b, n, d, beta, alpha, x);
    }
    free(Y); free(z); free(d); free(idx);
    return 0;
}

int oracle_sgd(const double *X, int64_t ld, int64_t m, int64_t n, const double *y,
               double *x, double eta, double lambda, int32_t b, uint64_t seed,
               uint64_t step0, int64_t nsteps)
{
    rows_t R = {X, 0, ld};
    return sgd_impl(R, m, n, y, NULL, x, eta, lambda, b, seed, step0, nsteps, LOSS_LOGISTIC);
}

int oracle_sgd_glm(const double *X, int64_t ld, int64_t m, int64_t n, const double *y,
                   double *x, double eta, double lambda, int32_t b, uint64_t seed,
                   uint64_t step0, int64_t nsteps, int32_t loss)
{
    rows_t R = {X, 0, ld};
    return sgd_impl(R, m, n, y, NULL, x, eta, lambda, b, seed, step0, nsteps, loss);
}

int oracle_sgd_f32(const float *X, int64_t ld, int64_t m, int64_t n, const float *y,
                   double *x, double eta, double lambda, int32_t b, uint64_t seed,
                   uint64_t step0, int64_t nsteps)
{
    rows_t R = {X, 1, ld};
    return sgd_impl(R, m, n, NULL, y, x, eta, lambda, b, seed, step0, nsteps, LOSS_LOGISTIC);
}

int oracle_sgd_glm_f32(const float *X, int64_t ld, int64_t m, int64_t n, const float *y,
                       double *x, double eta, double lambda, int32_t b, uint64_t seed,
                       uint64_t step0, int64_t nsteps, int32_t loss)
{
    rows_t R = {X, 1, ld};
    return sgd_impl(R, m, n, NULL, y, x, eta, lambda, b, seed, step0, nsteps, loss);
}

/* One s-step outer iteration's data-dependent pieces for rows Y (sb x n):
 * r = Y x and the strict block-lower part of G = Y Y^T (other entries 0). */
static void margin_and_gram(const double *Y, int32_t b, int32_t s, int64_t n,
                            const double *x, double *r, double *G)
{
    const int64_t sb = (int64_t)s * b;
    rows_times_x(Y, sb, n, x, r);
    memset(G, 0, sizeof(double) * (size_t)sb * (size_t)sb);
#pragma omp parallel for schedule(dynamic, 1) if (sb * sb * n > OMP_MIN_WORK)
    for (int64_t t = 0; t < sb; ++t) {
        int64_t j = t / b;
        for (int64_t u = 0; u < j * b; ++u) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += Y[t * n + k] * Y[u * n + k];
            G[t * sb + u] = acc;
        }
    }
}

/* The s inner residual corrections (Algorithm 1, inner loop, with decay).
 * Inputs r[sb], G (strict block-lower, row-major sb x sb), labels yI[sb].
 * Outputs delta[sb] and c[sb] = beta^(s-1-j) delta for rows of block j. */
static void inner_corrections(const double *G, const double *r, const double *yI,
                              int32_t b, int32_t s, double alpha, double beta,
                              double *delta, double *c, int loss)
{
    const int64_t sb = (int64_t)s * b;
    for (int32_t j = 0; j < s; ++j) {
        const double bj = pow(beta, (double)j);
        for (int32_t q = 0; q < b; ++q) {
            const int64_t t = (int64_t)j * b + q;
            double acc = 0.0;
            for (int32_t i = 0; i < j; ++i) {
                const double w = pow(beta, (double)(j - 1 - i));
                double part = 0.0;
                for (int32_t p = 0; p < b; ++p)
                    part += G[t * sb + (int64_t)i * b + p] * delta[(int64_t)i * b + p];
                acc += w * part;
            }
            const double z = bj * r[t] + alpha * acc;
            delta[t] = glm_delta(z, yI[t], loss);
        }
    }
    for (int32_t j = 0; j < s; ++j) {
        const double w = pow(beta, (double)(s - 1 - j));
        for (int32_t q = 0; q < b; ++q)
            c[(int64_t)j * b + q] = w * delta[(int64_t)j * b + q];
    }
}

int oracle_inner_corrections(const double *G, const double *r, const double *yI,
                             int32_t b, int32_t s, double eta, double lambda,
                             double *delta, double *c)
{
    inner_corrections(G, r, yI, b, s, eta / (double)b, 1.0 - eta * lambda, delta, c,
                      LOSS_LOGISTIC);
    return 0;
}

int oracle_inner_corrections_glm(const double *G, const double *r, const double *yI,
                                 int32_t b, int32_t s, double eta, double lambda,
                                 double *delta, double *c, int32_t loss)
{
    inner_corrections(G, r, yI, b, s, eta / (double)b, 1.0 - eta * lambda, delta, c, loss);
    return 0;
}

typedef struct {
    int64_t *idx;
    double *Y, *r, *G, *yI, *delta, *c;
} outer_ws;

static int ws_alloc(outer_ws *w, int64_t sb, int64_t n)
{
    w->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)sb);
    w->Y = (double *)malloc(sizeof(double) * (size_t)sb * (size_t)n);
    w->r = (double *)malloc(sizeof(double) * (size_t)sb);
    w->G = (double *)malloc(sizeof(double) * (size_t)sb * (size_t)sb);
    w->yI = (double *)malloc(sizeof(double) * (size_t)sb);
    w->delta = (double *)malloc(sizeof(double) * (size_t)sb);
    w->c = (double *)malloc(sizeof(double) * (size_t)sb);
    return (w->idx && w->Y && w->r && w->G && w->yI && w->delta && w->c) ? 0 : -3;
}

static void ws_free(outer_ws *w)
{
    free(w->idx); free(w->Y); free(w->r); free(w->G);
    free(w->yI); free(w->delta); free(w->c);
}

static int casgd_impl(rows_t X, int64_t m, int64_t n, const double *y,
                      const float *y32, double *x, double eta, double lambda,
                      int32_t b, int32_t s, uint64_t seed, uint64_t outer0,
                      int64_t nouter, int loss)
{
    if (m <= 0 || n <= 0 || b <= 0 || s <= 0)
        return -1;
    const int64_t sb = (int64_t)s * b;
    const double alpha = eta / (double)b;
    const double beta = 1.0 - eta * lambda;
    const double beta_s = pow(beta, (double)s);
    outer_ws w;
    if (ws_alloc(&w, sb, n)) {
        ws_free(&w);
        return -3;
    }
    for (int64_t hh = 0; hh < nouter; ++hh) {
        uint64_t h = outer0 + (uint64_t)hh;
        oracle_sample_indices(seed, h * (uint64_t)sb, sb, m, w.idx);
        gather_rows(X, n, w.idx, sb, w.Y);
        for (int64_t q = 0; q < sb; ++q)
            w.yI[q] = y ? y[w.idx[q]] : (double)y32[w.idx[q]];
        margin_and_gram(w.Y, b, s, n, x, w.r, w.G);
        inner_corrections(w.G, w.r, w.yI, b, s, alpha, beta, w.delta, w.c, loss);
        decay_plus_yt_w(w.Y, sb, n, w.c, beta_s, alpha, x);
    }
    ws_free(&w);
    return 0;
}

int oracle_casgd(const double *X, int64_t ld, int64_t m, int64_t n, const double *y,
                 double *x, double eta, double lambda, int32_t b, int32_t s,
                 uint64_t seed, uint64_t outer0, int64_t nouter)
{
    rows_t R = {X, 0, ld};
    return casgd_impl(R, m, n, y, NULL, x, eta, lambda, b, s, seed, outer0, nouter,
                      LOSS_LOGISTIC);
}

int oracle_casgd_glm(const double *X, int64_t ld, int64_t m, int64_t n, const double *y,
                     double *x, double eta, double lambda, int32_t b, int32_t s,
                     uint64_t seed, uint64_t outer0, int64_t nouter, int32_t loss)
{
    rows_t R = {X, 0, ld};
    return casgd_impl(R, m, n, y, NULL, x, eta, lambda, b, s, seed, outer0, nouter, loss);
}

int oracle_casgd_f32(const float *X, int64_t ld, int64_t m, int64_t n,
                     const float *y, double *x, double eta, double lambda,
                     int32_t b, int32_t s, uint64_t seed, uint64_t outer0,
                     int64_t nouter)
{
    rows_t R = {X, 1, ld};
    return casgd_impl(R, m, n, NULL, y, x, eta, lambda, b, s, seed, outer0, nouter,
                      LOSS_LOGISTIC);
}

int oracle_casgd_glm_f32(const float *X, int64_t ld, int64_t m, int64_t n,
                         const float *y, double *x, double eta, double lambda,
                         int32_t b, int32_t s, uint64_t seed, uint64_t outer0,
                         int64_t nouter, int32_t loss)
{
    rows_t R = {X, 1, ld};
    return casgd_impl(R, m, n, NULL, y, x, eta, lambda, b, s, seed, outer0, nouter, loss);
}

/* The pieces of outer iteration `outer` from the current x, for per-step
 * comparisons: sampled indices, labels, r, strict block-lower G, and the
 * recurrence outputs delta and c. x is not modified. */
int oracle_outer_parts_glm(const double *X, int64_t ld, int64_t m, int64_t n,
                           const double *y, const double *x, double eta, double lambda,
                           int32_t b, int32_t s, uint64_t seed, uint64_t outer,
                           int64_t *idx_out, double *yI_out, double *r_out,
                           double *G_out, double *delta_out, double *c_out, int32_t loss)
{
    if (m <= 0 || n <= 0 || b <= 0 || s <= 0)
        return -1;
    const int64_t sb = (int64_t)s * b;
    double *Y = (double *)malloc(sizeof(double) * (size_t)sb * (size_t)n);
    if (!Y)
        return -3;
    rows_t R = {X, 0, ld};
    oracle_sample_indices(seed, outer * (uint64_t)sb, sb, m, idx_out);
    gather_rows(R, n, idx_out, sb, Y);
    for (int64_t q = 0; q < sb; ++q)
        yI_out[q] = y[idx_out[q]];
    margin_and_gram(Y, b, s, n, x, r_out, G_out);
    inner_corrections(G_out, r_out, yI_out, b, s, eta / (double)b, 1.0 - eta * lambda,
                      delta_out, c_out, loss);
    free(Y);
    return 0;
}

/* One outer iteration on given sampled rows Y (sb x n, row-major) with their
 * labels yI: Algorithm 1 after the sampling and gather steps (margins, strict
 * block-lower Gram, inner corrections, update). Writes r, G, delta, c and the
 * new iterate x_out (n); x is not modified. */
int oracle_outer_rows_glm(const double *Y, int64_t n, const double *yI, const double *x,
                          double eta, double lambda, int32_t b, int32_t s,
                          double *r_out, double *G_out, double *delta_out, double *c_out,
                          double *x_out, int32_t loss)
{
    if (n <= 0 || b <= 0 || s <= 0)
        return -1;
    const int64_t sb = (int64_t)s * b;
    const double alpha = eta / (double)b;
    const double beta = 1.0 - eta * lambda;
    margin_and_gram(Y, b, s, n, x, r_out, G_out);
    inner_corrections(G_out, r_out, yI, b, s, alpha, beta, delta_out, c_out, loss);
    memcpy(x_out, x, sizeof(double) * (size_t)n);
    decay_plus_yt_w(Y, sb, n, c_out, pow(beta, (double)s), alpha, x_out);
    return 0;
}

int oracle_outer_parts(const double *X, int64_t ld, int64_t m, int64_t n,
                       const double *y, const double *x, double eta, double lambda,
                       int32_t b, int32_t s, uint64_t seed, uint64_t outer,
                       int64_t *idx_out, double *yI_out, double *r_out,
                       double *G_out, double *delta_out, double *c_out)
{
    return oracle_outer_parts_glm(X, ld, m, n, y, x, eta, lambda, b, s, seed, outer, idx_out,
                                  yI_out, r_out, G_out, delta_out, c_out, LOSS_LOGISTIC);
}

/* ------------------------------------------------------------- CSR rows */

/* Sparse dot of two rows with sorted column indices. */
static double sparse_dot(const int32_t *ca, const double *va, int64_t na,
                         const int32_t *cb, const double *vb, int64_t nb)
{
    double acc = 0.0;
    int64_t p = 0, q = 0;
    while (p < na && q < nb) {
        if (ca[p] == cb[q]) {
            acc += va[p] * vb[q];
            ++p; ++q;
        } else if (ca[p] < cb[q]) {
            ++p;
        } else {
            ++q;
        }
    }
    return acc;
}

/* s-step SGD on a CSR matrix (column indices sorted within each row). Same
 * arithmetic as the dense version with the zero entries skipped; the sums
 * visit the stored entries in column order. */
int oracle_casgd_csr_glm(const int64_t *row_ptr, const int32_t *col_idx, const double *val,
                         int64_t m, int64_t n, const double *y, double *x, double eta,
                         double lambda, int32_t b, int32_t s, uint64_t seed,
                         uint64_t outer0, int64_t nouter, int32_t loss)
{
    if (m <= 0 || n <= 0 || b <= 0 || s <= 0)
        return -1;
    const int64_t sb = (int64_t)s * b;
    const double alpha = eta / (double)b;
    const double beta = 1.0 - eta * lambda;
    const double beta_s = pow(beta, (double)s);
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)sb);
    double *r = (double *)malloc(sizeof(double) * (size_t)sb);
    double *G = (double *)malloc(sizeof(double) * (size_t)sb * (size_t)sb);
    double *yI = (double *)malloc(sizeof(double) * (size_t)sb);
    double *d = (double *)malloc(sizeof(double) * (size_t)sb);
    double *c = (double *)malloc(sizeof(double) * (size_t)sb);
    double *g = (double *)calloc((size_t)n, sizeof(double));
    if (!idx || !r || !G || !yI || !d || !c || !g) {
        free(idx); free(r); free(G); free(yI); free(d); free(c); free(g);
        return -3;
    }
    for (int64_t hh = 0; hh < nouter; ++hh) {
        uint64_t h = outer0 + (uint64_t)hh;
        oracle_sample_indices(seed, h * (uint64_t)sb, sb, m, idx);
        for (int64_t t = 0; t < sb; ++t) {
            int64_t i = idx[t];
            yI[t] = y[i];
            double acc = 0.0;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                acc += val[p] * x[col_idx[p]];
            r[t] = acc;
        }
        memset(G, 0, sizeof(double) * (size_t)sb * (size_t)sb);
#pragma omp parallel for schedule(dynamic, 4) if (sb > 256)
        for (int64_t t = 0; t < sb; ++t) {
            int64_t j = t / b, it = idx[t];
            for (int64_t u = 0; u < j * b; ++u) {
                int64_t iu = idx[u];
                G[t * sb + u] = sparse_dot(col_idx + row_ptr[it], val + row_ptr[it],
                                           row_ptr[it + 1] - row_ptr[it],
                                           col_idx + row_ptr[iu], val + row_ptr[iu],
                                           row_ptr[iu + 1] - row_ptr[iu]);
            }
        }
        inner_corrections(G, r, yI, b, s, alpha, beta, d, c, loss);
        /* x <- beta^s x + alpha * Y^T c: accumulate Y^T c column by column in
         * sample order, then apply. */
        memset(g, 0, sizeof(double) * (size_t)n);
        for (int64_t t = 0; t < sb; ++t) {
            int64_t i = idx[t];
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                g[col_idx[p]] += val[p] * c[t];
        }
        for (int64_t k = 0; k < n; ++k)
            x[k] = beta_s * x[k] + alpha * g[k];
    }
    free(idx); free(r); free(G); free(yI); free(d); free(c); free(g);
    return 0;
}

int oracle_casgd_csr(const int64_t *row_ptr, const int32_t *col_idx, const double *val,
                     int64_t m, int64_t n, const double *y, double *x, double eta,
                     double lambda, int32_t b, int32_t s, uint64_t seed,
                     uint64_t outer0, int64_t nouter)
{
    return oracle_casgd_csr_glm(row_ptr, col_idx, val, m, n, y, x, eta, lambda, b, s, seed,
                                outer0, nouter, LOSS_LOGISTIC);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from now on (timing the oracle on one core). */
void oracle_set_threads(int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}
