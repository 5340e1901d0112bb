/*
 * hsp_oracle.c -- plain FP64 CPU oracle of the Horseshoe Probit Gibbs sweep.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares no
 * code, header or constant table with the GPU library.
 *
 * Reference: Terenin, Dong & Draper, "GPU-accelerated Gibbs sampling: a case
 * study of the Horseshoe Probit model".  Equation and section numbers below
 * refer to that paper.  Every step is the plain definition, one loop at a
 * time, in double precision.  The only places where float32 appears are the
 * three accept/branch decisions of the truncated-normal sampler, which are
 * taken in float32 on purpose (the paper's GPU arithmetic), so that both this
 * oracle and the GPU kernel decide on the same side of each threshold.
 *
 * Parity status of each part (how it is pinned by the tests):
 *   Philox4x32-10        pinned: bit-identical to rocRAND's independent engine
 *   uniform map          pinned: exact values, open interval, moments
 *   truncated normal     pinned: closed-form TN moments, KS, acceptance rates,
 *                        sign invariant, 0.47 crossover of Section 5
 *   Cheng gamma          pinned: moments, KS, closed-form acceptance 1/M
 *   exponential draws    pinned: KS against the exponential law
 *   Cholesky / solves    pinned: LAPACK (numpy) and scipy triangular solves
 *   beta conditional     pinned: explicit-inverse mean and covariance,
 *                        chi-square Mahalanobis law
 *   whole sweep          pinned: X = 0 reduces to the half-Cauchy prior;
 *                        p = 2 grid posterior with lambda, tau frozen;
 *                        recovery of the nonzero coefficients (Section 6.1)
 */
#include "hsp_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads for the N-sized loops (the z step, X^T z, the Gram).  Each loop is
 * split so that every sum keeps its sequential order, so the results are the
 * same bits for any number of threads. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011), the counter-based      */
/* generator the paper recommends for per-thread skip-ahead (Section 5).    */
/* Ten rounds; each round multiplies counter words 0 and 2 by two fixed     */
/* 32-bit constants, mixes high halves with the other words and the key,    */
/* and the key is advanced by two Weyl increments between rounds.           */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Open-interval uniform: the top 23 bits of w, made odd, scaled by 2^-24. */
double orc_uniform(uint32_t w)
{
    return (2.0 * (double)(w >> 9) + 1.0) * (1.0 / 16777216.0);
}

void orc_words(uint64_t seed, uint32_t c0, uint32_t sweep, uint32_t tag,
               uint32_t round, uint32_t chain, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, sweep, (tag << 24) | (round & 0x00FFFFFFu), chain};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* The pair of uniforms of attempt a (two attempts per Philox call). */
static void attempt_uniforms(uint64_t seed, uint32_t c0, uint32_t sweep, uint32_t tag,
                             uint32_t chain, uint32_t a, double* u1, double* u2)
{
    uint32_t w[4];
    orc_words(seed, c0, sweep, tag, a >> 1, chain, w);
    if ((a & 1u) == 0) { *u1 = orc_uniform(w[0]); *u2 = orc_uniform(w[1]); }
    else               { *u1 = orc_uniform(w[2]); *u2 = orc_uniform(w[3]); }
}

/* ------------------------------------------------------------------------ */
/* Truncated normal z ~ TN(eta, 1, y), Section 5, z step ii:                */
/*   y* = 2y - 1, mu* = y* eta; draw t ~ N(mu*, 1) restricted to t > 0 and  */
/*   return z = y* t.                                                       */
/*   mu* > 0.47: Gaussian rejection, t = mu* + n, accept if t > 0.          */
/*   otherwise : Robert (1995) exponential rejection with the optimal rate  */
/*               for the lower bound -mu* of w = t - mu*:                   */
/*               theta = (-mu* + sqrt(mu*^2 + 4)) / 2,                      */
/*               t = -ln(u1) / theta,  accept if u2 < exp(-(w - theta)^2/2).*/
/* ------------------------------------------------------------------------ */
double orc_tn_draw(double eta, int y, uint64_t seed, uint32_t row, uint32_t sweep,
                   uint32_t chain, int32_t max_attempts, int32_t* attempt, int32_t* branch)
{
    const double ystar = y ? 1.0 : -1.0;
    const double mu = ystar * eta;
    const int gauss = (float)mu > 0.47f;
    const double theta = (-mu + sqrt(mu * mu + 4.0)) / 2.0;
    if (branch) *branch = gauss ? ORC_BRANCH_GAUSS : ORC_BRANCH_ROBERT;
    for (int32_t a = 0; a < max_attempts; ++a) {
        double u1, u2;
        attempt_uniforms(seed, row, sweep, ORC_TAG_Z, chain, (uint32_t)a, &u1, &u2);
        if (gauss) {
            /* Box-Muller normal from (u1, u2). */
            double n = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
            double t = mu + n;
            if ((float)t > 0.0f) {
                if (attempt) *attempt = a;
                return ystar * t;
            }
        } else {
            double t = -log(u1) / theta;
            double w = t - mu;
            double rho = exp(-(w - theta) * (w - theta) / 2.0);
            if ((float)u2 < (float)rho) {
                if (attempt) *attempt = a;
                return ystar * t;
            }
        }
    }
    if (attempt) *attempt = -1;
    return NAN;
}

/* ------------------------------------------------------------------------ */
/* Gamma(a, 1) by Cheng (1977), algorithm GB, for a > 1 (Section 5, tau^-2  */
/* step iii).  Proposal: the log-logistic law with exponent                 */
/* lambda = sqrt(2a - 1) and median a, sampled by inversion:                */
/*   V = ln(u1 / (1 - u1)) / lambda,  X = a e^V.                            */
/* Accept if  (a - ln 4) + (a + lambda) V - X >= ln(u1^2 u2); a cheaper     */
/* squeeze accepts first when the left side plus 1 + ln 4.5 - 4.5 u1^2 u2  */
/* is nonnegative.  Attempt m uses the uniforms of round m/2 of tag TAU.    */
/* ------------------------------------------------------------------------ */
double orc_gamma_cheng(double a, uint64_t seed, uint32_t sweep, uint32_t chain,
                       int32_t* attempt)
{
    const double A = 1.0 / sqrt(2.0 * a - 1.0);
    const double B = a - log(4.0);
    const double C = a + 1.0 / A;
    const double D = 1.0 + log(4.5);
    for (int32_t m = 0; m < (1 << 24); ++m) {
        double u1, u2;
        attempt_uniforms(seed, 0, sweep, ORC_TAG_TAU, chain, (uint32_t)m, &u1, &u2);
        double V = A * log(u1 / (1.0 - u1));
        double X = a * exp(V);
        double Z = u1 * u1 * u2;
        double R = B + C * V - X;
        if (R + D - 4.5 * Z >= 0.0 || R >= log(Z)) {
            if (attempt) *attempt = m;
            return X;
        }
    }
    if (attempt) *attempt = -1;
    return NAN;
}

/* ------------------------------------------------------------------------ */
/* Element access: float32, or bfloat16 bits widened exactly to float.      */
/* ------------------------------------------------------------------------ */
static double xval(const void* X, int xtype, int64_t idx)
{
    if (xtype == ORC_X_BF16) {
        uint32_t bits = (uint32_t)((const uint16_t*)X)[idx] << 16;
        float f;
        memcpy(&f, &bits, sizeof f);
        return (double)f;
    }
    return (double)((const float*)X)[idx];
}

double orc_row_dot(const void* X, int xtype, int64_t p, int64_t row, const double* beta)
{
    double s = 0.0;
    for (int64_t j = 0; j < p; ++j) s += xval(X, xtype, row * p + j) * beta[j];
    return s;
}

/* z step (Section 5): eta = X beta, then one TN draw per row.  The rows are
 * full-conditionally independent (Eq. 8), so any order gives the same z. */
void orc_z_step(const void* X, int xtype, const uint8_t* y, int64_t N, int64_t p,
                const double* beta, uint64_t seed, uint32_t sweep, uint32_t chain,
                double* z, int32_t* attempt, int32_t* branch)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double eta = orc_row_dot(X, xtype, p, i, beta);
        int32_t a = 0, br = 0;
        z[i] = orc_tn_draw(eta, y[i] ? 1 : 0, seed, (uint32_t)i, sweep, chain, 1 << 16, &a, &br);
        if (attempt) attempt[i] = a;
        if (branch) branch[i] = br;
    }
}

/* b_j = sum_i x_ij z_i, summed over i in order.  Threads own blocks of 64
 * columns (each still summed row by row, in order). */
void orc_xtz(const void* X, int xtype, int64_t N, int64_t p, const double* z, double* b)
{
    const int64_t nblk = (p + 63) / 64;
#pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < nblk; ++blk) {
        const int64_t j0 = 64 * blk, j1 = j0 + 64 < p ? j0 + 64 : p;
        for (int64_t j = j0; j < j1; ++j) b[j] = 0.0;
        for (int64_t i = 0; i < N; ++i)
            for (int64_t j = j0; j < j1; ++j) b[j] += xval(X, xtype, i * p + j) * z[i];
    }
}

/* G_jk = sum_i x_ij x_ik, summed over i in order; threads own rows j of G. */
void orc_gram(const void* X, int xtype, int64_t N, int64_t p, double* G)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < p; ++j) {
        for (int64_t k = 0; k < p; ++k) G[j * p + k] = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double xj = xval(X, xtype, i * p + j);
            for (int64_t k = 0; k < p; ++k) G[j * p + k] += xj * xval(X, xtype, i * p + k);
        }
    }
}

double orc_gram_entry(const void* X, int xtype, int64_t N, int64_t p, int64_t j, int64_t k)
{
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += xval(X, xtype, i * p + j) * xval(X, xtype, i * p + k);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Exponential draws by inversion, -ln(u)/rate (Section 5, lambda/nu/xi     */
/* steps; rate parameterisation fixed by Eq. 11).                           */
/* ------------------------------------------------------------------------ */
static double exp_draw(double rate, uint64_t seed, uint32_t idx, uint32_t sweep,
                       uint32_t tag, uint32_t chain)
{
    uint32_t w[4];
    orc_words(seed, idx, sweep, tag, 0, chain, w);
    return -log(orc_uniform(w[0])) / rate;
}

int64_t orc_lambda_step(int64_t p, const double* beta, const double* nu_m1, double tau_m2,
                        uint64_t seed, uint32_t sweep, uint32_t chain, double* lam_m2)
{
    int64_t clamps = 0;
    for (int64_t j = 0; j < p; ++j) {
        double rate = nu_m1[j] + tau_m2 * beta[j] * beta[j] / 2.0;
        if (!(rate >= DBL_MIN)) { rate = DBL_MIN; ++clamps; }
        lam_m2[j] = exp_draw(rate, seed, (uint32_t)j, sweep, ORC_TAG_LAMBDA, chain);
    }
    return clamps;
}

double orc_tau_step(int64_t p, const double* lam_m2, const double* beta, double xi_m1,
                    uint64_t seed, uint32_t sweep, uint32_t chain, int32_t* attempt)
{
    double sum = 0.0;
    for (int64_t j = 0; j < p; ++j) sum += lam_m2[j] * beta[j] * beta[j];
    double rate = xi_m1 + sum / 2.0;
    double shape = ((double)p + 1.0) / 2.0;
    double g = orc_gamma_cheng(shape, seed, sweep, chain, attempt);
    return g / rate;
}

void orc_nu_step(int64_t p, const double* lam_m2, uint64_t seed, uint32_t sweep,
                 uint32_t chain, double* nu_m1)
{
    for (int64_t j = 0; j < p; ++j)
        nu_m1[j] = exp_draw(1.0 + lam_m2[j], seed, (uint32_t)j, sweep, ORC_TAG_NU, chain);
}

double orc_xi_step(double tau_m2, uint64_t seed, uint32_t sweep, uint32_t chain)
{
    return exp_draw(1.0 + tau_m2, seed, 0, sweep, ORC_TAG_XI, chain);
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra, textbook forms.                                    */
/* ------------------------------------------------------------------------ */
/* Q = U^T U, U upper, row by row:
 *   U_jj = sqrt(Q_jj - sum_{k<j} U_kj^2),
 *   U_ji = (Q_ji - sum_{k<j} U_kj U_ki) / U_jj   (i > j),
 * each sum taken in the order k = 0, 1, ..., j-1.  The entries of one row j
 * depend only on rows above it, so they are computed on OpenMP threads; the
 * factor is built in a work array holding U^T row-major (column j of U is a
 * contiguous row there), which changes where the values sit, not what is
 * summed or in which order. */
int orc_cholesky_upper(int64_t p, const double* Q, double* U)
{
    double* Lt = (double*)calloc((size_t)(p * p), sizeof(double)); /* Lt[i p + k] = U_ki */
    int rc = 0;
    for (int64_t j = 0; j < p && rc == 0; ++j) {
        const double* uj = Lt + j * p;
        double d = Q[j * p + j];
        for (int64_t k = 0; k < j; ++k) d -= uj[k] * uj[k];
        if (!(d > 0.0)) {
            rc = (int)(j + 1);
            break;
        }
        const double ujj = sqrt(d);
        Lt[j * p + j] = ujj;
#pragma omp parallel for schedule(static) if (p - j > 256)
        for (int64_t i = j + 1; i < p; ++i) {
            const double* ui = Lt + i * p;
            double s = Q[j * p + i];
            for (int64_t k = 0; k < j; ++k) s -= uj[k] * ui[k];
            Lt[i * p + j] = s / ujj;
        }
    }
    for (int64_t r = 0; r < p; ++r)
        for (int64_t c = 0; c < p; ++c) U[r * p + c] = c >= r ? Lt[c * p + r] : 0.0;
    free(Lt);
    return rc;
}

void orc_solve_upper(int64_t p, const double* U, const double* r, double* x)
{
    for (int64_t i = p - 1; i >= 0; --i) {
        double s = r[i];
        for (int64_t k = i + 1; k < p; ++k) s -= U[i * p + k] * x[k];
        x[i] = s / U[i * p + i];
    }
}

void orc_solve_upper_t(int64_t p, const double* U, const double* r, double* x)
{
    for (int64_t i = 0; i < p; ++i) {
        double s = r[i];
        for (int64_t k = 0; k < i; ++k) s -= U[k * p + i] * x[k];
        x[i] = s / U[i * p + i];
    }
}

/* beta step, Section 5 steps ii-viii:
 *   Q = X^T X + tau^-2 Lambda^-2;  Q = U^T U;  s ~ N(0, I);  U v = s
 *   (so Cov(v) = Q^-1);  U^T w = b, U mu = w (so mu = Q^-1 b);  beta = mu + v. */
int orc_beta_step(int64_t p, const double* G, const double* lam_m2, double tau_m2,
                  const double* b, uint64_t seed, uint32_t sweep, uint32_t chain,
                  double* beta, double* mean, double* noise)
{
    double* Q = (double*)malloc(sizeof(double) * (size_t)(p * p));
    double* U = (double*)malloc(sizeof(double) * (size_t)(p * p));
    double* s = (double*)malloc(sizeof(double) * (size_t)p);
    double* v = (double*)malloc(sizeof(double) * (size_t)p);
    double* w = (double*)malloc(sizeof(double) * (size_t)p);
    double* mu = (double*)malloc(sizeof(double) * (size_t)p);
    int rc = 0;
    for (int64_t k = 0; k < p * p; ++k) Q[k] = G[k];
    for (int64_t j = 0; j < p; ++j) Q[j * p + j] += tau_m2 * lam_m2[j];
    rc = orc_cholesky_upper(p, Q, U);
    if (rc == 0) {
        for (int64_t j = 0; j < p; ++j) {
            uint32_t wd[4];
            orc_words(seed, (uint32_t)j, sweep, ORC_TAG_BETA_S, 0, chain, wd);
            double u1 = orc_uniform(wd[0]), u2 = orc_uniform(wd[1]);
            s[j] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
        }
        orc_solve_upper(p, U, s, v);
        orc_solve_upper_t(p, U, b, w);
        orc_solve_upper(p, U, w, mu);
        for (int64_t j = 0; j < p; ++j) beta[j] = mu[j] + v[j];
        if (mean) memcpy(mean, mu, sizeof(double) * (size_t)p);
        if (noise) memcpy(noise, v, sizeof(double) * (size_t)p);
    }
    free(Q); free(U); free(s); free(v); free(w); free(mu);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Whole sweeps.                                                            */
/* ------------------------------------------------------------------------ */
void orc_cold_start(int64_t p, orc_state* s)
{
    for (int64_t j = 0; j < p; ++j) { s->beta[j] = 0.0; s->lam_m2[j] = 1.0; s->nu_m1[j] = 1.0; }
    s->tau_m2 = 1.0;
    s->xi_m1 = 1.0;
    s->sweep = 0;
}

int orc_sweep(const void* X, int xtype, const uint8_t* y, int64_t N, int64_t p,
              const double* G, uint64_t seed, uint32_t chain, orc_state* s,
              double* z_out, double* b_out, int64_t* clamps)
{
    const uint32_t k = s->sweep + 1;
    double* z = z_out ? z_out : (double*)malloc(sizeof(double) * (size_t)N);
    double* b = b_out ? b_out : (double*)malloc(sizeof(double) * (size_t)p);
    double* lam_new = (double*)malloc(sizeof(double) * (size_t)p);
    int rc;

    /* (i) z and lambda^-2 (both from the previous beta, nu, tau), then tau^-2
     * from the new lambda^-2. */
    orc_z_step(X, xtype, y, N, p, s->beta, seed, k, chain, z, NULL, NULL);
    int64_t c = orc_lambda_step(p, s->beta, s->nu_m1, s->tau_m2, seed, k, chain, lam_new);
    if (clamps) *clamps += c;
    memcpy(s->lam_m2, lam_new, sizeof(double) * (size_t)p);
    s->tau_m2 = orc_tau_step(p, s->lam_m2, s->beta, s->xi_m1, seed, k, chain, NULL);

    /* (ii) beta from the new z, lambda, tau; nu^-1 and xi^-1 from the new
     * lambda and tau. */
    orc_xtz(X, xtype, N, p, z, b);
    rc = orc_beta_step(p, G, s->lam_m2, s->tau_m2, b, seed, k, chain, s->beta, NULL, NULL);
    orc_nu_step(p, s->lam_m2, seed, k, chain, s->nu_m1);
    s->xi_m1 = orc_xi_step(s->tau_m2, seed, k, chain);
    s->sweep = k;

    if (!z_out) free(z);
    if (!b_out) free(b);
    free(lam_new);
    return rc;
}

int orc_run(const void* X, int xtype, const uint8_t* y, int64_t N, int64_t p,
            const double* G, uint64_t seed, uint32_t chain, orc_state* s, int64_t n,
            double* beta_draws, double* tau_draws, double* lam_draws)
{
    double* z = (double*)malloc(sizeof(double) * (size_t)N);
    double* b = (double*)malloc(sizeof(double) * (size_t)p);
    int rc = 0;
    for (int64_t t = 0; t < n && rc == 0; ++t) {
        rc = orc_sweep(X, xtype, y, N, p, G, seed, chain, s, z, b, NULL);
        if (beta_draws) memcpy(beta_draws + t * p, s->beta, sizeof(double) * (size_t)p);
        if (tau_draws) tau_draws[t] = s->tau_m2;
        if (lam_draws) memcpy(lam_draws + t * p, s->lam_m2, sizeof(double) * (size_t)p);
    }
    free(z);
    free(b);
    return rc;
}
