/*
 * hsp.h -- C ABI of the MI355X (gfx950) Horseshoe Probit Gibbs sampler.
 *
 * The library runs the data-parallel Gibbs sweep of Terenin, Dong & Draper,
 * "GPU-accelerated Gibbs sampling: a case study of the Horseshoe Probit
 * model", Section 5, for the model of Eqs. (9)-(10):
 *     y_i = 1{z_i > 0},  z_i ~ N(x_i beta, 1),
 *     beta_j ~ N(0, lambda_j^2 tau^2),  lambda_j, tau ~ C+(0, 1),
 * using the auxiliary-variable conditionals of Eq. (12).  One sweep is
 *   (i)  z | beta (N truncated normals around X beta, Eq. 8 makes them
 *        independent) in parallel with lambda^-2, followed by tau^-2;
 *   (ii) beta | z, lambda, tau (X^T z and a Cholesky solve of
 *        Q = X^T X + tau^-2 Lambda^-2, then a Gaussian draw), with nu^-1 and
 *        xi^-1 alongside.
 *
 * All arithmetic runs in the library's HIP kernels.  N-sized work (X beta,
 * the truncated-normal draws, X^T z) runs in float32 over X stored as
 * float32 or bfloat16; everything p-sized (X^T X, Q, its Cholesky factor,
 * the solves and the hyperparameters) runs in float64.
 *
 * Random numbers: Philox4x32-10 with key = seed and counter
 * (index, sweep number k >= 1, tag << 24 | round, chain id).  A state's
 * draws are a pure function of (X, y, seed, chain id, starting state), so
 * runs are bit-reproducible and resumable.  (The library stores column j of
 * X multiplied by 2^-e_j, the power of two that brings its largest
 * magnitude into (1/2, 1]; an exact scaling that leaves every product
 * x_ij beta_j unchanged.  X^T z is accumulated from float32 sums over a few
 * rows, each rounded to a multiple of 2^-24 in those column units, where
 * float64 sums are exact in any order, so the GPU's dynamic split of rows
 * between blocks does not change it and its rounding follows each column's
 * scale.  Exactness holds while sum_i |z_i| < 2^29; beyond that the results
 * keep float64 accuracy but may differ in the last bits between runs.
 * Entries below 2^-126 of their column's largest magnitude lose precision
 * to float32 subnormals.)
 *
 * Conventions shared by every entry point:
 *  - Every call returns an hsp_status and never aborts or throws.
 *  - Pointers named "device" must be HIP device (or managed) memory of the
 *    current device; "host" pointers are ordinary host memory.  The library
 *    never keeps a caller pointer beyond the call that receives it.
 *  - Matrices are row-major and dense unless stated otherwise.
 *  - After HSP_EHIP, HSP_ENOTPD or HSP_ERANGE reported by a sweep, the
 *    state is poisoned: later calls return HSP_EPOISONED until
 *    hsp_destroy.  hsp_last_error() describes the failure.
 *  - One state may be used by one host thread at a time.  Independent
 *    states may be used concurrently.
 */
#ifndef HSP_H
#define HSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsp_state hsp_state; /* opaque, owned by the library */

typedef enum {
    HSP_OK = 0,
    HSP_EINVAL = -1,    /* invalid argument or input data */
    HSP_ENOMEM = -2,    /* device or host allocation failed */
    HSP_EHIP = -3,      /* a HIP runtime call failed */
    HSP_ENOTPD = -4,    /* X^T X + tau^-2 Lambda^-2 was not positive definite */
    HSP_ERANGE = -5,    /* a draw left the representable range (NaN/inf) or the
                           requested draws are no longer stored */
    HSP_EPOISONED = -6  /* an earlier device failure poisoned this state */
} hsp_status;

typedef enum { HSP_X_F32 = 0, HSP_X_BF16 = 1 } hsp_xtype;

/* Options of hsp_create; hsp_default_options() fills the defaults. */
typedef struct {
    uint64_t seed;          /* Philox key (default 1) */
    uint32_t chain_id;      /* Philox counter word 3 (default 0) */
    int32_t x_type;         /* storage of X: HSP_X_F32 (default) or HSP_X_BF16
                               (rounded to nearest even at creation) */
    int32_t x_on_host;      /* 1: X and y are host pointers; 0 (default): device */
    int32_t record_lambda;  /* 1: also record lambda^-2 with every kept draw */
    int64_t thin;           /* keep the draw of every thin-th sweep (default 1) */
    int64_t max_draws;      /* capacity of the device-resident draw ring
                               (default 1024); older draws are overwritten */
    void* hip_stream;       /* hipStream_t to run on; NULL: the library's own */
    int32_t debug_store_z;  /* 1: keep z, the accepted attempt and X^T z of the
                               last z step for hsp_get_debug (costs N*8 bytes
                               of writes per sweep) */
    int32_t use_graph;      /* 1 (default): replay sweeps from a captured HIP graph */
    int32_t multi_chain_z;  /* batches: 1 (default) = chains sharing a bfloat16 design
                               with rows of at most 1024 elements run one z pass for
                               up to 16 of them (X beta and X^T z as matrix-core
                               products); 0 = every chain its own z pass */
    int32_t autotune;       /* 1: pick the launch shapes by measurement (see below);
                               0 (default): the built-in shapes */
    int32_t x_stream;       /* 1: keep the library's copy of X in pinned host memory
                               and stream it through the GPU in row chunks every
                               sweep (designs larger than device memory); 0 (default):
                               X resident in device memory */
    int64_t stream_rows;    /* with x_stream: rows per chunk (rounded to the row
                               splits of the one-time X^T X); 0 (default): about
                               256 MB of X per chunk */
} hsp_options;

void hsp_default_options(hsp_options* opt);

/*
 * Autotuning.  With autotune = 1, hsp_create (and hsp_batch_create's first
 * hsp_batch_sweep) picks how the sweep kernel splits its work -- the blocks
 * of the p-side group, and how the z pass deals out its row tiles (a share
 * statically, the rest in claimed units); for a batch, the blocks of each
 * multi-chain z pass, how many chains share a launch, and the balance of
 * z-pass and p-side blocks in those launches -- by timing a few sweeps of
 * each candidate on the device.  The
 * chain's state is restored afterwards, and no choice changes any draw:
 * a tuned chain draws bit for bit what an untuned one draws.  If the
 * environment variable HSP_TUNE_CACHE names a file, a choice found there for
 * the same device, shape and library is used without measuring, and new
 * choices are added to it (a text file of "key<TAB>value" lines).
 */

/*
 * Create a sampler state from the design X (N x p float32, row-major,
 * leading dimension p) and outcomes y (N bytes, each 0 or 1).
 * X and y are read during the call only; the library keeps its own copy
 * (rows padded to 16 bytes, converted to bfloat16 if requested).  Computes
 * G = X^T X once in float64 (Section 5, beta step i) and sets the cold start
 * of Section 6.1 (beta = 0; lambda = nu = tau = xi = 1).
 * With x_stream, the library's copy of X lives in pinned host memory and
 * every sweep streams it through two device chunk buffers (copies on a
 * stream of their own, overlapped with the z pass of the previous chunk);
 * the chain draws bit for bit what a resident chain draws whenever the row
 * splits of X^T X are the same (always when about 256 MB of X holds one
 * split).  Throughput is then bound by the host-to-device link.
 * Errors: HSP_EINVAL if N < 2, p < 2, N >= 2^32, p > hsp_max_p(), a y_i is
 * not 0/1 or an X entry is not finite; HSP_ENOMEM; HSP_EHIP.
 */
hsp_status hsp_create(const float* X, const uint8_t* y, int64_t N, int64_t p,
                      const hsp_options* opt, hsp_state** out);

/* Largest p the library supports. */
int64_t hsp_max_p(void);

/*
 * G = X^T X in float64 (Section 5, beta step i: the one-time product the
 * precision matrix Q = X^T X + tau^-2 Lambda^-2 is built from) for a design
 * on the device.  X: N x p, row-major with leading dimension ld >= p
 * elements, float32 (x_type HSP_X_F32) or bfloat16 bit patterns (HSP_X_BF16,
 * uint16 per element); every element is widened exactly to float64 and the
 * products are summed on the FP64 matrix cores in a fixed order (the same G,
 * bit for bit, on every call).  G: device buffer of p x p doubles, row-major,
 * written whole (symmetric).  Allocates a device workspace of about
 * 32 KB x (64-wide tile pairs of G) x (row splits) and frees it before
 * returning; runs on hip_stream (NULL: the null stream) and waits for it.
 * Errors: HSP_EINVAL (NULL pointers, N < 1, p < 1, ld < p, N or ld >= 2^32,
 * unknown x_type); HSP_ENOMEM; HSP_EHIP.
 */
hsp_status hsp_gram(const void* X, int32_t x_type, int64_t N, int64_t p, int64_t ld, double* G,
                    void* hip_stream);

/*
 * hsp_gram without any allocation, for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc).  Same arguments, same result bit for bit as hsp_gram.  The
 * partial tiles go to a fixed workspace of 32 MiB compiled into the library
 * (one per device, held until the process ends) instead of a fresh buffer;
 * large G are processed in several rounds through it.  Every call on one
 * device shares that workspace, so calls that overlap in time on one device
 * (other host threads, or other streams) race and must not be issued.
 * Runs on hip_stream (NULL: the null stream) and waits for it.
 * Errors: as hsp_gram; HSP_EINVAL also if a single 64 x 64 tile's partials
 * (32 KB per row split; at most 1024 splits on a 256-CU device) exceed the
 * workspace.
 */
hsp_status hsp_gram_noalloc(const void* X, int32_t x_type, int64_t N, int64_t p, int64_t ld,
                            double* G, void* hip_stream);

/*
 * Enqueue n_iter full sweeps on the state's stream and return without
 * waiting.  Sweep k draws, in order: z and lambda^-2 from beta^(k-1), then
 * tau^-2; then beta, nu^-1 and xi^-1 (Section 5, updates (i)-(ii)), and
 * records beta, tau^-2 (and lambda^-2 if requested) when k is a multiple of
 * thin.  Device failures surface at the next synchronising call.
 * Errors: HSP_EINVAL if n_iter < 0; HSP_EPOISONED; HSP_EHIP.
 */
hsp_status hsp_sweep(hsp_state* s, int64_t n_iter);

/* Wait for the state's enqueued work and report device failures
 * (HSP_ENOTPD, HSP_ERANGE). */
hsp_status hsp_sync(hsp_state* s);

/*
 * The Monte-Carlo output (Section 5: the draws of each iteration are
 * written out while the next iterations run, so the GPU never waits on the
 * host).  Here the kept draws stay in a device-resident ring (288 GB of HBM
 * hold long chains) and are copied out on request.
 * Copy kept draws [first, first + count) (0-based, in recording order since
 * creation or the last hsp_set_state) into host buffers: beta (count x p),
 * tau_m2 (count), lam_m2 (count x p, only if record_lambda, else may be
 * NULL).  Synchronises first.  *n_out receives the number of draws recorded
 * so far.  Errors: HSP_ERANGE if a requested draw was overwritten or not yet
 * recorded; device failures as hsp_sync.
 */
hsp_status hsp_draws(hsp_state* s, double* beta, double* tau_m2, double* lam_m2,
                     int64_t first, int64_t count, int64_t* n_out);

/*
 * Reorder the library's copy of the rows of X (and y) by y*_i x_i beta of
 * the current state, y* = 2y - 1 (Section 5 suggests it after burn-in, so
 * that rows whose truncated normals take the same branch and accept after
 * similar numbers of proposals share a wave).  Every row keeps its Philox
 * counters and its place in hsp_get_debug's outputs, so z is drawn exactly
 * as before; X^T z is then summed over other groups of rows, so b and the
 * chain change within float32 rounding.  Allocates a second copy of X while
 * it runs.  Synchronises.  Errors: HSP_EINVAL for a streamed state or a
 * chain of a batch; HSP_ENOMEM; HSP_EHIP; HSP_EPOISONED.
 */
hsp_status hsp_sort_rows(hsp_state* s);

/* Release every resource of the state (waits for its work first).  A chain
 * of a batch is released with its batch (HSP_EINVAL here). */
hsp_status hsp_destroy(hsp_state* s);

/* Text of the last failure on this state (never NULL); for a NULL state,
 * the last failure of hsp_create on this thread. */
const char* hsp_last_error(const hsp_state* s);

/* ---- Batches: many independent chains, one graph launch per sweep ----------
 * (A batch is its own handle, hsp_batch, created by hsp_batch_create; its
 * chains are reached as ordinary hsp_state handles through hsp_batch_chain,
 * so every state entry point applies to them.)
 * A batch runs chains of the same sweep on several designs at once (the
 * chains of one design share its library copy of X, y and G = X^T X).  One
 * hsp_batch_sweep advances every chain by the same number of sweeps; each
 * batched sweep is a single replay of a captured HIP graph holding every
 * chain's sweep kernel, one after another on the batch's stream (the
 * multi-chain passes described below may run on a second stream beside the
 * other chains' launches; the graph joins it before their p-side launch).
 * Every dataset of a batch is resident (x_stream is ignored).  Chain i
 * (dataset-major order) uses Philox counter word 3 = opt->chain_id + i, so it
 * draws exactly what a lone sampler created with that chain id draws --
 * except chains that share a bfloat16 design under multi_chain_z: their
 * X beta and X^T z run as bfloat16 matrix-core products with beta and z
 * split into two bfloat16 parts each (error <= 2^-18 relative per term, then
 * float32 accumulation), and for p > 16 their beta comes from blocked
 * substitution through the Cholesky factor (their factorisation runs beside
 * or after the pass, not under a pass of their own, and leaves L^-1 out).
 * They follow the same conditionals and counters, are bit-reproducible run
 * to run, but round differently from a lone chain. */
typedef struct hsp_batch hsp_batch; /* opaque, owned by the library */

typedef struct {
    const float* X;   /* N x p float32, row-major (device, or host if x_on_host) */
    const uint8_t* y; /* N bytes, each 0 or 1 */
    int64_t N;
    int64_t p;
    int32_t x_type;   /* storage of this X: HSP_X_F32 or HSP_X_BF16 */
} hsp_dataset;

/* Create chains_per_ds[d] chains on each of the n_ds datasets (read during
 * the call only, as in hsp_create).  opt gives the options of every chain
 * (its x_type is ignored: each dataset states its own; its hip_stream, if
 * set, is the batch's stream).  Errors: as hsp_create for any dataset;
 * HSP_EINVAL if n_ds < 1, a count is < 1 or the total exceeds 65536. */
hsp_status hsp_batch_create(const hsp_dataset* ds, int32_t n_ds, const int32_t* chains_per_ds,
                            const hsp_options* opt, hsp_batch** out);
/* Number of chains. */
int64_t hsp_batch_size(const hsp_batch* b);
/* A borrowed handle of chain i, valid until hsp_batch_destroy: every state
 * entry point accepts it (hsp_draws, hsp_get_state, ...), hsp_destroy does not. */
hsp_status hsp_batch_chain(hsp_batch* b, int64_t i, hsp_state** chain);
/* Enqueue n_iter sweeps of every chain and return without waiting.
 * Errors: HSP_EINVAL if n_iter < 0; HSP_EPOISONED if a chain is poisoned; HSP_EHIP. */
hsp_status hsp_batch_sweep(hsp_batch* b, int64_t n_iter);
/* Wait for the batch's work and report the first chain's device failure. */
hsp_status hsp_batch_sync(hsp_batch* b);
/* Timing of the batched sweeps enqueued while enabled (a pair of HIP events
 * on the batch's stream around each graph replay, at most 256 pairs in use
 * as for hsp_set_timing): mean ms per batched sweep. */
hsp_status hsp_batch_set_timing(hsp_batch* b, int32_t enable);
hsp_status hsp_batch_get_timing(hsp_batch* b, double* ms_per_sweep, int64_t* n_sweeps);
/* Text of the batch's last failure (never NULL; NULL batch: the last failed
 * creation on this thread). */
const char* hsp_batch_last_error(const hsp_batch* b);
/* Release the batch and all its chains (waits for its work first). */
hsp_status hsp_batch_destroy(hsp_batch* b);

/* ---- Markov state: checkpoint / resume and test hooks --------------------- */
/* Copy the Markov state to host buffers (beta, lam_m2, nu_m1: p doubles;
 * any pointer may be NULL).  Synchronises; a device failure found while
 * synchronising poisons the state, hence the non-const handle. */
hsp_status hsp_get_state(hsp_state* s, double* beta, double* lam_m2, double* nu_m1,
                         double* tau_m2, double* xi_m1, uint64_t* sweep);
/* Overwrite the Markov state from host buffers; sweep is the number of
 * completed sweeps (the next sweep uses counter k = sweep + 1).  Resets the
 * draw count.  Errors: HSP_EINVAL for a negative or non-finite entry of
 * lam_m2, nu_m1, tau_m2, xi_m1 or a non-finite beta. */
hsp_status hsp_set_state(hsp_state* s, const double* beta, const double* lam_m2,
                         const double* nu_m1, double tau_m2, double xi_m1, uint64_t sweep);

/* Steps for hsp_step (bitmask). */
enum {
    HSP_STEP_Z = 1,       /* z | beta and b = X^T z (Section 5, z step; beta step vi) */
    HSP_STEP_LAMBDA = 2,  /* lambda^-2 | beta, nu, tau */
    HSP_STEP_TAU = 4,     /* tau^-2 | lambda, beta, xi */
    HSP_STEP_BETA = 8,    /* beta | b, lambda, tau (Section 5, beta steps ii-viii) */
    HSP_STEP_NUXI = 16,   /* nu^-1 | lambda and xi^-1 | tau */
    HSP_STEP_ADVANCE = 32 /* then count the sweep as completed */
};
/* Run the selected conditionals once, in the sweep's order, with counter
 * k = (completed sweeps) + 1, without recording a draw.  Synchronises. */
hsp_status hsp_step(hsp_state* s, uint32_t which);

/* Debug outputs of the last z step (needs debug_store_z): z (N floats),
 * attempt (N int32: 0-based index of the accepted proposal, up to 4095, with
 * bit 30 set when the row took the Gaussian branch; 32 bits hold both), b =
 * X^T z (p doubles).  NULL skips an output. */
hsp_status hsp_get_debug(hsp_state* s, float* z, int32_t* attempt, double* b);

/* G = X^T X (p x p doubles, host). */
hsp_status hsp_get_gram(hsp_state* s, double* G);

/* Counters since creation: number of lambda rates clamped up to DBL_MIN and
 * the largest number of truncated-normal proposals any row needed. */
hsp_status hsp_get_counters(hsp_state* s, uint64_t* lambda_clamps, uint32_t* max_attempts);

/* Timing of the sweeps enqueued by hsp_sweep while enabled, measured with a
 * pair of HIP events on the state's stream around each sweep's launch:
 * zpass_ms = mean milliseconds per launch of the sweep kernel (z pass and
 * p-side share it), sweep_ms = (first start to last end) / sweeps.  Enabling
 * (hsp_set_timing(s, 1)) resets the counts.  At most 256 event pairs are in
 * use: when they are, hsp_sweep waits for the oldest timed sweeps and adds
 * their durations to a running sum. */
hsp_status hsp_set_timing(hsp_state* s, int32_t enable);
hsp_status hsp_get_timing(hsp_state* s, double* zpass_ms, double* sweep_ms, int64_t* n_sweeps);

#ifdef __cplusplus
}
#endif
#endif
