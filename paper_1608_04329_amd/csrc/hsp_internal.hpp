// Internal declarations shared by the library's HIP sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace hsp {

// Pointers that device code reads from memory (the launch description) lose
// their address space: qualifying them as global in the device pass keeps
// every access a global (not flat) memory instruction.  The layout is the
// same in both passes (64-bit pointers).
#if defined(__HIP_DEVICE_COMPILE__)
#define HSP_GLOBAL __attribute__((address_space(1)))
#else
#define HSP_GLOBAL
#endif

// The launch description itself is read-only for a whole launch: device code
// reaches it through the constant address space, which lets the compiler keep,
// hoist and re-load its fields freely (as it does for kernel arguments) across
// the kernel's atomics and fences.
#if defined(__HIP_DEVICE_COMPILE__)
#define HSP_CONST __attribute__((address_space(4)))
#else
#define HSP_CONST
#endif

// Host side: a device pointer as stored in a launch description.
template <class T>
inline HSP_GLOBAL T* dev_ptr(T* p) {
    return (HSP_GLOBAL T*)p;
}

constexpr int kWave = 64;
constexpr int kMaxP = 10240;           // largest p
constexpr uint32_t kLargeP = 4096;     // beyond this p the factorisation outweighs the pass over X
constexpr uint32_t kMaxRounds = 2048;  // 4096 truncated-normal proposals per row
constexpr int kThreads = 256;          // threads per block of the sweep kernel
constexpr int kTile = 64;              // p-side tile edge
constexpr int kSmallP = 16;            // p up to this runs the one-block p-side path
#ifndef HSP_MAX_GROUP
#define HSP_MAX_GROUP 48
#endif
constexpr int kMaxGroup = HSP_MAX_GROUP;  // most blocks of the p-side group
constexpr int kZGroup = 16;            // z-pass blocks whose partials one block sums
// The z pass for rows of kc 16-byte chunks per lane of a wave (xtype 0:
// float32, 4 elements per chunk; 1: bfloat16, 8): whether each wave holds
// whole rows (up to 1536 float32 or 1024 bfloat16 elements) or the row is
// split over the block's four waves, and the rows per tile.  Both are set by
// the register budget of two blocks per compute unit: a taller tile or a
// whole wider row in one wave spills.  Short rows get tall tiles (32 rows up
// to 256 float32 elements, 16 up to 512 float32 or bfloat16 elements): a
// tile's loads and its truncated-normal draws (one lane per row) then cover
// more rows at once.
constexpr bool wide_chunks(int xtype, int kc) { return xtype == 0 ? kc > 6 : kc > 2; }
constexpr int rows_for(int xtype, int kc) {
    if (!wide_chunks(xtype, kc)) return kc == 1 && xtype == 0 ? 32 : kc <= (xtype == 0 ? 2 : 1) ? 16 : kc <= 4 ? 8 : 4;
    const int kcw = (kc + 3) / 4;  // chunks per lane of each wave's quarter
    return xtype == 0 ? (kcw <= 3 ? 4 : kcw <= 7 ? 2 : 1) : (kcw <= 2 ? 4 : kcw <= 4 ? 2 : 1);
}
// How the z pass deals out its row tiles (a launch parameter; the autotuner
// may pick others): this share in percent statically, interleaved over all
// waves, the rest in units of this many tiles to whichever block asks next.
// Neither changes any result (X^T z is exact in any split of the rows).
constexpr uint32_t kZStaticPctDefault = 40;
constexpr uint32_t kZUnitDefault = 8;
constexpr uint32_t kZUnitMax = 64;
// LDS of one sweep-kernel block: two 64 x 66 float64 tiles (67,584 bytes; rows
// 16-byte aligned).  The same buffer holds the z pass's reduction segment and
// the packed Q of the one-block path (p (p + 1) / 2 <= 8256 doubles).
constexpr int kTileLd = kTile + 2;
constexpr int kLdsDoubles = 2 * kTile * kTileLd;

// Device control block, one per sampler state.  The counters that blocks
// poll or update concurrently each have a 128-byte line of their own.
struct Ctrl {
    uint32_t sweep;             // completed sweeps; sweep k uses counter k = sweep + 1
    uint32_t draw_base;         // value of sweep at creation or the last set_state
    uint32_t max_attempts;      // most proposals any row needed
    int32_t chol_info;          // first non-positive pivot (1-based), 0 if none
    unsigned long long clamps;  // lambda rates clamped to DBL_MIN
    unsigned long long bar_epoch;  // bar_count when the current launch started
    unsigned long long z_epoch;    // z_count when the current launch started
    alignas(128) uint32_t err;     // kErr* bits
    alignas(128) unsigned long long bar_count;  // arrivals at p-side group barriers (monotonic)
    alignas(128) unsigned long long z_count;    // z-pass groups finished (monotonic)
    alignas(128) uint32_t task_next;  // next factorisation task of the shared queue (zero between launches)
    alignas(128) uint32_t z_next;     // next z-pass unit of the shared remainder (zero between launches)
    alignas(128) uint32_t z_done;     // z groups finished in a launch without a p-side (zero between launches)
};

enum : uint32_t {
    kErrTnCap = 1u,      // a truncated-normal row hit the proposal cap (NaN input)
    kErrNotPD = 2u,      // non-positive pivot in the Cholesky factorisation
    kErrNonFinite = 4u,  // a p-sized draw became NaN or infinite
    kErrInput = 8u,      // invalid y or non-finite X at creation
    kErrTimeout = 16u,   // a bounded wait inside the sweep kernel gave up
};

// Work selected for one launch of the sweep kernel.
enum : uint32_t {
    kModeZ = 1u,         // z pass and b = X^T z
    kModeLambda = 2u,
    kModeTau = 4u,
    kModeBeta = 8u,
    kModeNuXi = 16u,
    kModeRecord = 32u,   // write the draw of this sweep into the ring
    kModeAdvance = 64u,  // count the sweep as completed
    kModeBsum = 128u,    // b = X^T z from bsum, accumulated by an earlier launch (no z pass here)
    // the tile path's p-side in two launches of one sweep (p > 16 only):
    kModePre = 256u,     // lambda, tau, nu, xi, the noise of beta and the factorisation, then stop
    kModePost = 512u,    // only what needs b: beta from the factorisation of the earlier launch
};

// Layout of X in device memory: row-major, leading dimension ld elements,
// ld a multiple of 16 bytes, padding columns zero.  Column j is stored
// multiplied by 2^-e_j, e_j chosen so that its largest magnitude lies in
// (1/2, 1]: the library's X is X D with D = diag(2^-e_j), an exact scaling.
// The z pass then runs on X D and beta D^-1 (the same products x_ij beta_j,
// bit for bit) and its X^T z comes out as D X^T z, so the fixed grid on
// which tile sums are rounded is 2^-24 of each column's own scale.
struct XLayout {
    HSP_GLOBAL const void* X;
    int xtype;  // 0 float32, 1 bfloat16
    uint32_t N;
    uint32_t p;
    uint32_t ld;
};

struct PackQ;

// Everything one launch of the sweep kernel touches.
struct SweepArgs {
    XLayout x;
    HSP_GLOBAL const uint8_t* y;
    HSP_GLOBAL float* beta32;      // ld floats (padding zero): beta_j 2^e_j for the z pass
    HSP_GLOBAL const double* xscale;  // p: 2^e_j, the scale of column j of the stored X
    HSP_GLOBAL double* partial;    // gz x ld: per-block float64 partials of X^T z
    HSP_GLOBAL double* bsum;       // ld: X^T z accumulated by the z groups (zero between launches)
    HSP_GLOBAL uint32_t* zgrp_count;  // zgroups arrival counters (zero between launches)
    HSP_GLOBAL float* zdbg;        // optional: z of the last z pass (N)
    HSP_GLOBAL int32_t* adbg;      // optional: accepted proposal | gauss bit (N)
    HSP_GLOBAL double* beta;       // p
    HSP_GLOBAL double* lam_m2;     // p
    HSP_GLOBAL double* nu_m1;      // p
    HSP_GLOBAL double* tau_m2;     // 1
    HSP_GLOBAL double* xi_m1;      // 1
    HSP_GLOBAL double* b;          // p: X^T z of the current sweep
    HSP_GLOBAL const double* G;    // p x p Gram
    HSP_GLOBAL const double* Gp;   // tile path: P x P, G with an identity block on the padding
    HSP_GLOBAL double* A;          // tile path, P x P: U (P = p rounded up to 64)
    HSP_GLOBAL double* Linv;       // tile path, P x P: lower triangle holds L^-1 = U^-T
    HSP_GLOBAL double* vec;        // 2 p scratch
    HSP_GLOBAL double* ring_beta;  // capacity x p
    HSP_GLOBAL double* ring_tau;   // capacity
    HSP_GLOBAL double* ring_lam;   // capacity x p or null
    uint32_t thin;
    uint32_t capacity;
    HSP_GLOBAL Ctrl* ctrl;
    uint64_t seed;
    uint32_t chain;
    uint32_t mode;           // kMode* bits
    uint32_t gp;             // blocks of the p-side group (first in the grid)
    uint32_t gz;             // z-pass blocks (after the group)
    uint32_t zgroups;        // ceil(gz / kZGroup)
    uint32_t block0;         // first grid block of this chain (several chains share a pack launch)
    uint32_t idle;           // a grid block that leaves at once (0: none), see sweep_finish_args
    uint64_t timeout_ticks;  // bound of every wait, in s_memrealtime ticks
    HSP_GLOBAL uint64_t* trace;         // optional: kTraceSlots timestamps per group block
    HSP_GLOBAL const uint32_t* tasks;   // tile path: every group block's task list, concatenated
    HSP_GLOBAL const uint32_t* task_off;  // gp + 1 offsets into tasks
    HSP_GLOBAL uint32_t* ver;           // tile path: 2 x nt x nt tile version counters (zero between launches)
    uint32_t z_static_pct;   // z pass: share of the row tiles dealt out statically (0..100)
    uint32_t z_unit;         // z pass: tiles per claimed unit of the rest (1..kZUnitMax)
    uint32_t first_row;      // global index of x.X's first row (X streamed in row chunks; else 0):
                             // y, the Philox counters and the debug outputs use global rows
    HSP_GLOBAL const uint32_t* row_id;  // original index of each stored row (rows reordered), or null
    HSP_GLOBAL PackQ* zq;  // the pack's shared z queue, or null (then gz blocks of its own)
    uint32_t subst;        // tile path: beta by blocked substitution (factorisation without L^-1)
};

// ---- the shared z queue of a pack -----------------------------------------------
// A pack may give its chains no z-pass blocks of their own: its worker
// blocks then take every chain's z pass from one queue.  Chain c's rows are
// cut into units[c] units of z_unit row tiles, claimed from next[c]; a worker
// drains the units of its home chain first, then those of whichever chain
// has most left.  When a worker leaves a chain it adds its float64 tile sums
// into the chain's b accumulator (exact on the 2^-24 grid, so the order of
// the additions does not matter) and then the number of units it finished
// into the chain's z_count, which the chain's p-side waits to reach
// zgroups = units[c].  A chain's draws are those of the chain alone.
constexpr int kPackQMax = 256;             // chains of a queue pack
constexpr uint16_t kWorkerBit = 0x8000u;   // block map: a worker of the queue (low bits: home chain)
struct PackQ {
    uint32_t nchains;
    uint32_t workers;                         // worker blocks of the launch
    alignas(128) uint32_t done;               // workers finished (zero between launches)
    alignas(128) uint32_t next[kPackQMax];    // next unit of each chain (zero between launches)
    alignas(128) uint32_t units[kPackQMax];   // units of each chain
};

// Device view of a launch description.
using Args = const HSP_CONST SweepArgs;

// ---- the multi-chain z pass (several chains sharing one bfloat16 design) ----------
// One pass over X serves up to kMcChains chains: X beta and X^T z for all of
// them are bfloat16 matrix-core products (beta and z split into a high and a
// low bfloat16 part each, float32 accumulation).  The four waves of a block
// split the columns of a tile of kMcRows rows; each wave holds up to kMcKs
// 32-column steps, so ld <= 4 * 32 * kMcKs.
constexpr int kMcChains = 16;
constexpr int kMcKs = 8;
constexpr int kMcRows = 16;
constexpr int kMcUnit = 64;  // tiles per claimed unit; each unit's X^T z is rounded to the grid
constexpr uint32_t kMcMaxLd = 4u * 32u * kMcKs;
// 32-column steps per wave of the pass for rows of ld elements, and the
// columns its four waves cover
inline uint32_t mc_steps(uint32_t ld) { return ld <= 4u * 32u * 4u ? 4u : (uint32_t)kMcKs; }
inline uint32_t mc_stride(uint32_t ld) { return 4u * 32u * mc_steps(ld); }

struct McArgs {
    XLayout x;                          // the shared design (bfloat16)
    HSP_GLOBAL const uint8_t* y;
    uint32_t nchains;                   // chains served (<= kMcChains)
    uint32_t gz;                        // blocks of the launch
    uint32_t zgroups;                   // ceil(gz / kZGroup)
    HSP_GLOBAL double* partial;         // gz x kMcChains x pstride float64 block partials of X^T z
    uint32_t pstride;                   // mc_stride(ld): every column a block's waves cover
    HSP_GLOBAL uint32_t* count;         // [0, zgroups): group arrivals; [zgroups]: groups done;
                                        // [zgroups + 32]: next unit (zero between launches)
    HSP_GLOBAL const SweepArgs* chain[kMcChains];  // the chains' launch descriptions
};

// Diagnostic trace per group block: slot 0 = start, slots 1.. one value per
// event in order (group barriers: a timestamp; per factorisation task: its
// index in the task array, then timestamps when its inputs were ready, loaded
// and done), then kTraceRecs records of kTraceRec slots for the diagonal tiles
// the block factored (loaded, panels, stored), and the last slot = z pass
// seen complete.
constexpr int kTraceSlots = 512;
constexpr int kTraceSeq = 448;
constexpr int kTraceRec = 12;
constexpr int kTraceRecs = 5;

// ---- tasks of the tiled factorisation (p > 16) ----------------------------------
enum : uint32_t { kTaskPotrf = 0u, kTaskTrsm = 1u, kTaskGemm = 2u, kTaskPanel = 3u };
// type (2 bits) | part (0: U, 1: L^-1) | step k | tile row i | tile column j (8 bits each)
constexpr uint32_t kTaskField = 255u;  // nt <= 255 tiles per side
__host__ __device__ constexpr uint32_t task_code(uint32_t type, uint32_t part, uint32_t k, uint32_t i,
                                                 uint32_t j) {
    return type | part << 2 | k << 3 | i << 11 | j << 19;
}
// Task lists of the factorisation of [Q | I] for a group of gp blocks
// (schedule.cpp): with gp = 1 one list, tasks[off[0] .. off[1]), run in order by
// block 0; with gp > 1 block 0's chain list tasks[off[0] .. off[1]) and the
// shared queue tasks[off[1] .. off[2]) the other blocks claim in order.
// Whether the factorisation of nt tiles per side carries L^-1 = U^-T along
// (beta as two parallel triangular products) or leaves it out beyond the
// diagonal tiles (beta by blocked substitution).  L^-1 is half of the
// factorisation's flops; up to p = kSubstP the factorisation hides under the
// z pass and the products make the shorter tail, beyond it the substitution's
// latency costs less (measured: N = 1e6, p = 1500: 1.10 ms per sweep with L^-1
// against 1.23 ms; N = 5e5, p = 2048: 1.66 against 1.29 ms; N = 2e5, p = 4096:
// 11.5 against 6.5 ms).
constexpr int kSubstP = 1536;
constexpr bool with_inverse(uint32_t nt) { return nt * (uint32_t)kTile <= (uint32_t)kSubstP; }
// inverse: whether the L^-1 tasks are part of the graph (a lone chain:
// with_inverse(nt); the chains of a multi-chain pass, whose factorisation
// does not hide under a pass of their own, leave them out)
void chol_schedule(uint32_t nt, uint32_t gp, std::vector<uint32_t>* tasks,
                   std::vector<uint32_t>* off, bool inverse);

struct SweepPlan {
    uint32_t gp;
    uint32_t gz;
    int chunks;    // 16-byte vectors per lane per row
    int rows;      // rows per wave tile
    int capacity;  // resident blocks of the chosen kernel on the device
    uint32_t cus = 0;  // compute units of the device
    uint32_t static_pct = kZStaticPctDefault;
    uint32_t unit = kZUnitDefault;
};

// Plan a launch for X's shape; num_cus from the device.  gp_req > 0 asks for
// a p-side group of that many blocks (clamped to what the shape can use);
// the z pass gets the rest of the resident capacity, up to one block per
// four row tiles.
hipError_t sweep_plan(const XLayout& x, int num_cus, SweepPlan* plan, uint32_t gp_req = 0);
// Largest p-side group a shape can use on a device of this capacity.
uint32_t max_group(const XLayout& x, int capacity);
// Fill gp, gz and zgroups of a launch description from the plan and its mode.
void sweep_finish_args(SweepArgs* a, const SweepPlan& plan);
// Enqueue one launch of the sweep kernel for one chain: table is a device
// array whose entry 0 points to a device copy of host.
hipError_t sweep_launch(const SweepArgs& host, const SweepArgs* const* table, const SweepPlan& plan,
                        hipStream_t st);
// Several chains in one launch (a pack): block b runs chain chain_of_block[b]
// (device arrays); every chain's description has its block0, gp and gz set.
// pack_capacity: resident blocks of that kernel on the device.
int pack_capacity(int xtype, int chunks, int num_cus);
hipError_t pack_launch(int xtype, int chunks, const SweepArgs* const* table, const uint16_t* chain_of_block,
                       uint32_t blocks, hipStream_t st);
// The multi-chain z pass over a shared bfloat16 design (mc: device copy of
// its description, gz blocks): every chain's X^T z is added into its bsum.
// The chains' p-side groups follow in a launch of their own with kModeBsum.
hipError_t mc_launch(const McArgs* mc, uint32_t ld, uint32_t gz, hipStream_t st);

// G = X^T X (p x p float64, leading dimension p) of the stored X, unscaled
// with the column exponents e (null: none).  The rows are cut into nsplit
// splits of rows_per_split rows and the upper triangle of G into npairs
// 64 x 64 tiles; every (split, tile) partial is summed in split order.
struct GramGeometry {
    uint32_t nt, npairs, nsplit, rows_per_split;
};
// max_rows_per_split > 0 caps the rows of a split (more splits), so that a
// design streamed in chunks of whole splits can form its partials chunk by chunk.
GramGeometry gram_geometry(const XLayout& x, int num_cus, uint64_t max_rows_per_split = 0);
// The partial tiles of every tile pair over the splits of one chunk of rows
// (chunk.N rows, the splits split0, split0 + 1, ... of geometry g, chunk.N a
// multiple of g.rows_per_split except for the last chunk) into work, which
// holds g.nsplit x g.npairs tiles; then G from all of them, summed in split
// order exactly as gram_launch sums them (the same G, bit for bit, when g is
// the same geometry).
hipError_t gram_chunk_launch(const XLayout& chunk, const GramGeometry& g, uint32_t split0, double* work,
                             hipStream_t st);
hipError_t gram_reduce_launch(const double* work, const GramGeometry& g, uint32_t p, const int32_t* e, double* G,
                              hipStream_t st);
// Doubles of workspace that hold every partial tile at once.
size_t gram_work_doubles(const XLayout& x, int num_cus);
// work must hold gram_work_doubles(x) doubles.
hipError_t gram_launch(const XLayout& x, const int32_t* e, double* G, double* work, int num_cus,
                       hipStream_t st);
// The same G (bit for bit) with a workspace of work_doubles doubles: the
// tiles are processed in chunks whose partials fit it (at least one tile's
// nsplit partials, else hipErrorInvalidValue).
hipError_t gram_launch_chunked(const XLayout& x, const int32_t* e, double* G, double* work,
                               size_t work_doubles, int num_cus, hipStream_t st);
// Doubles of workspace one 64 x 64 tile pair needs (its partials over every
// row split); gram_launch_chunked needs at least this much.
size_t gram_pair_doubles(const XLayout& x, int num_cus);
// The library's fixed Gram workspace (kGramScratchDoubles doubles, 32 MiB,
// one per device, held until the process ends): its device address on the
// current device.  Calls that use it on one device at the same time race.
constexpr size_t kGramScratchDoubles = (size_t)1 << 22;
hipError_t gram_scratch(double** ptr);
// Gp (P x P) = G with an identity block beyond p, zeros elsewhere.
hipError_t pad_gram_launch(const double* G, uint32_t p, uint32_t P, double* Gp, hipStream_t st);

// Input validation: sets kErrInput in ctrl if a y is not 0/1 or an X entry is
// not finite.
hipError_t validate_launch(const XLayout& x, const uint8_t* y, Ctrl* ctrl, hipStream_t st);

// Largest |x_ij| of every column of a float32 N x p matrix (leading dimension
// p): colmax_bits[j] receives the float bits of max_i |x_ij| (atomic maximum
// on the bit pattern; start from zeros).
hipError_t colmax_launch(const float* src, uint32_t N, uint32_t p, uint32_t* colmax_bits,
                         hipStream_t st);

// Copy / convert a float32 N x p matrix (leading dimension p) into the padded
// library layout, column j multiplied by 2^-e[j] (exact).  src may be the
// destination itself when the layouts coincide (float32, ld = p).
hipError_t pack_x_launch(const float* src, const XLayout& dst, const int32_t* e, hipStream_t st);

// Reordering the stored rows: key[i] = (2 y_i - 1) x_i beta (float32, the
// stored, column-scaled X with beta32), then Xo[i] = X[perm[i]], yo[i] =
// y[perm[i]], ido[i] = id ? id[perm[i]] : perm[i] (Xo, X: same layout).
hipError_t row_key_launch(const XLayout& x, const float* beta32, const uint8_t* y, float* key, hipStream_t st);
hipError_t gather_rows_launch(const XLayout& x, const uint32_t* perm, void* Xo, const uint8_t* y, uint8_t* yo,
                              const uint32_t* id, uint32_t* ido, hipStream_t st);

// Stream `bytes` of x with plain 16-byte loads only (the read ceiling).
hipError_t stream_read_launch(const void* x, size_t bytes, int num_cus, float* sink, hipStream_t st);

hipError_t philox_test_launch(uint64_t seed, const uint32_t* ctr, uint32_t n, uint32_t* out,
                              hipStream_t st);

}  // namespace hsp
