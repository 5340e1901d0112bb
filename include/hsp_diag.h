/*
 * hsp_diag.h -- diagnostic and test hooks of the Horseshoe Probit sampler
 * (include/hsp.h).  None of these is needed to run a chain: they expose the
 * device Philox generator (for bit-exactness tests), the factorisation's
 * task schedule (for its coverage and deadlock-freedom tests), a per-block
 * phase trace of the sweep kernel, a read-ceiling probe of the GPU, and the
 * autotuner's plan and cache.
 * Same conventions as hsp.h.
 */
#ifndef HSP_DIAG_H
#define HSP_DIAG_H

#include "hsp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Diagnostics: when enabled, every launch of the sweep kernel stores, per
 * block of its p-side group, a timestamp at the start (slot 0); then, in
 * order from slot 1 up to slot 447, one value per event: a timestamp for each
 * group barrier passed, and for each factorisation task (p > 16) its index
 * in the task lists of hsp_tile_schedule plus one, then timestamps of when its
 * inputs were ready, its input tiles were loaded and it was done; from slot
 * 448, five records of 12 slots for the diagonal tiles the block factored
 * (loaded, after each of the four panels and their updates, stored); and in
 * the last slot the moment the z pass was seen complete.
 * hsp_get_phase_trace copies group_blocks x slots uint64 values of the last
 * launch; ticks_per_us converts the timestamps.  Enabling drops the captured
 * graph. */
hsp_status hsp_set_phase_trace(hsp_state* s, int32_t enable);
hsp_status hsp_get_phase_trace(hsp_state* s, uint64_t* out, int64_t* group_blocks, int64_t* slots,
                               double* ticks_per_us);

/* The factorisation schedule for p > 16 (host only, no device work): the
 * Cholesky factorisation of Q by 64 x 64 tiles (Section 5, beta step iii),
 * with the same row operations applied to an identity block, is split into
 * tile tasks that the p-side blocks of the sweep kernel run.  nt =
 * ceil(p / 64) tiles per side, gp blocks; inverse: 1 with the L^-1 tasks,
 * 0 without them (beta then by blocked substitution), -1 as a lone chain of
 * that size has it (with them up to 24 tiles).
 * Task code: type (bits 0-1: 0 factor a diagonal tile, 1 triangular solve of
 * a tile of the block row, 2 tile update, 3 the next diagonal tile's solve,
 * update and factorisation in one block) | part (bit 2: 0 U, 1 L^-1) | step
 * k (bits 3-10) | tile row i (bits 11-18) | tile column j (bits 19-26).
 * With gp = 1, off[0..1] delimits block 0's list; with gp > 1, off[0..1]
 * delimits block 0's list (the critical chain) and off[1..2] the shared
 * queue that the other blocks claim tasks from, in order.  tasks (capacity
 * cap) receives the lists, off (3 entries) their bounds, *n_tasks the total
 * count (also when cap is too small, then HSP_ERANGE).  Errors: HSP_EINVAL
 * if nt < 1, nt > hsp_max_p() / 64, gp < 1 or inverse is not -1, 0 or 1.
 * Test hook for the schedule's coverage and deadlock freedom. */
hsp_status hsp_tile_schedule(int64_t nt, int64_t gp, int32_t inverse, uint32_t* tasks, int64_t cap,
                             uint32_t* off, int64_t* n_tasks);

/* Read ceiling of this GPU for the state's design: the mean milliseconds of
 * one pass of a plain streaming read (16-byte non-temporal loads, nothing
 * else) over the library's copy of X (N x ld elements), over `iters` passes
 * after two untimed ones, timed with HIP events on the state's stream.  The
 * z pass reads the same bytes; this bounds what it can reach.  Synchronises.
 * Errors: HSP_EINVAL if iters < 1; HSP_EPOISONED; HSP_EHIP. */
hsp_status hsp_read_ceiling(hsp_state* s, int32_t iters, double* ms_per_pass, double* bytes_per_pass);

/* Philox4x32-10 on the device: out[4i..4i+3] = Philox(ctr[4i..4i+3], key =
 * seed).  ctr and out are host arrays of 4n words.  Test hook for the
 * generator's bit-exactness. */
hsp_status hsp_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out);

/* The launch plan a state sweeps with: blocks of the p-side group and of the
 * z pass, the share of z-pass row tiles dealt out statically (percent) and
 * the tiles per claimed unit of the rest; note (capacity note_cap, may be
 * NULL) receives how the plan was chosen ("built-in", or the autotuner's
 * choice and whether it was measured or read from the cache). */
hsp_status hsp_get_plan(hsp_state* s, int64_t* group_blocks, int64_t* z_blocks, int64_t* static_pct,
                        int64_t* unit, char* note, int64_t note_cap);

/* The launch shapes of a batch's packs: blocks of each multi-chain z pass
 * (0: the built-in two per compute unit), the z-pass bandwidth per block that
 * the pack split model assumes (percent of nominal), the number of packs
 * (0 until the first hsp_batch_sweep), and how they were chosen (the note
 * also gives the most chains per pack the autotuner allowed). */
hsp_status hsp_batch_get_plan(hsp_batch* b, int64_t* mc_blocks, int64_t* bw_pct, int64_t* packs, char* note,
                              int64_t note_cap);

/* Two launch-shape choices of a batch (defaults 64 and 16), each leaving
 * every chain's draws bitwise those of the chain alone:
 *  - zq_kib: packs of chains with short rows (each row within one wave)
 *    take their z passes from one shared queue per pack, in units of about
 *    zq_kib KiB of X; 0 gives each chain z-pass blocks of its own;
 *  - pre_blocks: chains served by a multi-chain z pass (p > 16) draw lambda,
 *    tau, nu, xi and factor Q in a launch beside that pass, with this many
 *    blocks per chain; 0 does all of their p-side after the pass.
 * The packs are planned again at the next hsp_batch_sweep and the autotuner
 * is switched off for the batch.  HSP_EINVAL unless both lie in [0, 4096]. */
hsp_status hsp_batch_set_shape(hsp_batch* b, int32_t zq_kib, int32_t pre_blocks);

/* The autotuner's cache key of a state (its device, shape and plan format). */
hsp_status hsp_tune_key(hsp_state* s, char* key, int64_t cap);

/* The autotuner's cache file (host only, no device work): store value under
 * key (replacing an earlier entry of that key; keys hold no tab or newline,
 * values no newline), and read it back (HSP_ERANGE if absent). */
hsp_status hsp_tune_cache_put(const char* path, const char* key, const char* value);
hsp_status hsp_tune_cache_get(const char* path, const char* key, char* value, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif
