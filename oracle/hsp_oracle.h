/*
 * hsp_oracle.h -- plain FP64 CPU oracle of the Horseshoe Probit Gibbs sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  The product path never calls it and shares no code with it.
 *
 * Model and conditionals: Terenin, Dong & Draper, "GPU-accelerated Gibbs
 * sampling: a case study of the Horseshoe Probit model", Section 5,
 * Eqs. (9)-(12).  Every function below is written for clarity, one obvious
 * loop at a time, in double precision.
 *
 * Random numbers follow one counter contract shared (as a specification, not
 * as code) with the GPU library:
 *   generator : Philox4x32-10 (Salmon et al. 2011, recommended in Section 5)
 *   key       : (seed & 0xffffffff, seed >> 32)
 *   counter   : (c0 = row or coordinate index, c1 = sweep number k (1-based),
 *                c2 = tag << 24 | round, c3 = chain id)
 *   uniform   : u = (2*(w >> 9) + 1) * 2^-24, strictly inside (0,1) and exact
 *               in both float and double
 *   attempts  : one Philox call gives 4 words = 2 attempts; attempt a uses
 *               round a/2 and words (w0,w1) if a is even, (w2,w3) if odd
 */
#ifndef HSP_ORACLE_H
#define HSP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_TAG_Z = 1,       /* latent z_i draws                         */
    ORC_TAG_LAMBDA = 2,  /* lambda_j^-2 exponential draws            */
    ORC_TAG_TAU = 3,     /* tau^-2 gamma (Cheng) proposals           */
    ORC_TAG_BETA_S = 4,  /* standard normals s_j for the beta draw   */
    ORC_TAG_NU = 5,      /* nu_j^-1 exponential draws                */
    ORC_TAG_XI = 6       /* xi^-1 exponential draw                   */
};

enum { ORC_X_F32 = 0, ORC_X_BF16 = 1 };

/* Branch codes reported by orc_tn_draw. */
enum { ORC_BRANCH_ROBERT = 0, ORC_BRANCH_GAUSS = 1 };

/* Threads of the N-sized loops (OpenMP; results do not depend on it). */
void orc_set_threads(int n);
int  orc_max_threads(void);

/* ---- random numbers (Section 5, RNG discussion) ------------------------ */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint32_t w);
void   orc_words(uint64_t seed, uint32_t c0, uint32_t sweep, uint32_t tag,
                 uint32_t round, uint32_t chain, uint32_t out[4]);

/* ---- single draws -------------------------------------------------------- */
/* z ~ TN(eta, 1, y): Section 5, z step ii (a)-(c).  Returns z; reports the
 * 0-based index of the accepted attempt (-1 if max_attempts was reached, in
 * which case z is NaN) and the branch taken. */
double orc_tn_draw(double eta, int y, uint64_t seed, uint32_t row, uint32_t sweep,
                   uint32_t chain, int32_t max_attempts, int32_t* attempt, int32_t* branch);

/* Gamma(a, 1) by Cheng's (1977) algorithm GB, a > 1, drawing attempt m from
 * tag TAU, index 0.  Reports the 0-based accepted attempt. */
double orc_gamma_cheng(double a, uint64_t seed, uint32_t sweep, uint32_t chain,
                       int32_t* attempt);

/* ---- the conditionals of Eq. (12) -------------------------------------- */
/* z_i for every row, given beta (Section 5, z steps i-ii). X is N x p
 * row-major, float32 or bfloat16 bits.  attempt/branch may be NULL. */
void orc_z_step(const void* X, int xtype, const uint8_t* y, int64_t N, int64_t p,
                const double* beta, uint64_t seed, uint32_t sweep, uint32_t chain,
                double* z, int32_t* attempt, int32_t* branch);

/* eta_i = x_i . beta for one row (Section 5, z step i). */
double orc_row_dot(const void* X, int xtype, int64_t p, int64_t row, const double* beta);

/* b = X^T z (Section 5, beta step vi). */
void orc_xtz(const void* X, int xtype, int64_t N, int64_t p, const double* z, double* b);

/* G = X^T X (Section 5, beta step i), full p x p. */
void orc_gram(const void* X, int xtype, int64_t N, int64_t p, double* G);
/* One entry G_jk, summed over all rows in order. */
double orc_gram_entry(const void* X, int xtype, int64_t N, int64_t p, int64_t j, int64_t k);

/* lambda_j^-2 ~ Exp(nu_j^-1 + tau^-2 beta_j^2 / 2).  Returns the number of
 * rates clamped up to DBL_MIN. */
int64_t orc_lambda_step(int64_t p, const double* beta, const double* nu_m1, double tau_m2,
                        uint64_t seed, uint32_t sweep, uint32_t chain, double* lam_m2);

/* tau^-2 ~ Gamma(shape (p+1)/2, rate xi^-1 + sum_j lam_j^-2 beta_j^2 / 2). */
double orc_tau_step(int64_t p, const double* lam_m2, const double* beta, double xi_m1,
                    uint64_t seed, uint32_t sweep, uint32_t chain, int32_t* attempt);

/* nu_j^-1 ~ Exp(1 + lam_j^-2);  xi^-1 ~ Exp(1 + tau^-2). */
void   orc_nu_step(int64_t p, const double* lam_m2, uint64_t seed, uint32_t sweep,
                   uint32_t chain, double* nu_m1);
double orc_xi_step(double tau_m2, uint64_t seed, uint32_t sweep, uint32_t chain);

/* ---- dense linear algebra for the beta step ------------------------------ */
/* Q = U^T U with U upper triangular (row-major, lower part set to 0).
 * Returns 0, or j+1 if the pivot of column j is not positive. */
int  orc_cholesky_upper(int64_t p, const double* Q, double* U);
/* Solve U x = r (back substitution) and U^T x = r (forward substitution). */
void orc_solve_upper(int64_t p, const double* U, const double* r, double* x);
void orc_solve_upper_t(int64_t p, const double* U, const double* r, double* x);

/* beta ~ N(Q^-1 b, Q^-1), Q = G + tau^-2 diag(lam^-2) (Section 5, beta steps
 * ii-viii).  mean/noise (may be NULL) receive Q^-1 b and U^-1 s.
 * Returns 0 or the Cholesky failure code. */
int orc_beta_step(int64_t p, const double* G, const double* lam_m2, double tau_m2,
                  const double* b, uint64_t seed, uint32_t sweep, uint32_t chain,
                  double* beta, double* mean, double* noise);

/* ---- whole sweeps -------------------------------------------------------- */
typedef struct {
    double*  beta;    /* p */
    double*  lam_m2;  /* p */
    double*  nu_m1;   /* p */
    double   tau_m2;
    double   xi_m1;
    uint32_t sweep;   /* number of completed sweeps */
} orc_state;

/* Cold start of Section 6.1: beta = 0, lambda = nu = tau = xi = 1. */
void orc_cold_start(int64_t p, orc_state* s);

/* One sweep in the order of Section 5: (i) z and lambda^-2, then tau^-2;
 * (ii) beta, nu^-1 and xi^-1.  z, b (may be NULL) receive the sweep's latent
 * draws and X^T z.  Returns 0, or a Cholesky failure code. */
int orc_sweep(const void* X, int xtype, const uint8_t* y, int64_t N, int64_t p,
              const double* G, uint64_t seed, uint32_t chain, orc_state* s,
              double* z, double* b, int64_t* clamps);

/* n sweeps, recording beta (n x p), tau^-2 (n) and, if non-NULL, lam^-2. */
int orc_run(const void* X, int xtype, const uint8_t* y, int64_t N, int64_t p,
            const double* G, uint64_t seed, uint32_t chain, orc_state* s, int64_t n,
            double* beta_draws, double* tau_draws, double* lam_draws);

#ifdef __cplusplus
}
#endif
#endif
