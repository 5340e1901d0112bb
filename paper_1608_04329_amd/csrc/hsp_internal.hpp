// Internal declarations shared by the library's HIP sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsp {

constexpr int kWave = 64;
constexpr int kMaxP = 4096;          // largest p the register-tiled z pass supports
constexpr uint32_t kMaxRounds = 2048; // 4096 truncated-normal proposals per row

// Device control block, one per sampler state.
struct Ctrl {
    uint32_t sweep;          // completed sweeps; sweep k uses counter k = sweep + 1
    uint32_t draw_base;      // value of sweep at creation or the last set_state
    uint32_t err;            // kErr* bits
    uint32_t max_attempts;   // most proposals any row needed
    unsigned long long clamps;  // lambda rates clamped to DBL_MIN
    int32_t chol_info;       // first non-positive pivot (1-based), 0 if none
    uint32_t pad;
};

enum : uint32_t {
    kErrTnCap = 1u,      // a truncated-normal row hit the proposal cap (NaN input)
    kErrNotPD = 2u,      // non-positive pivot in the Cholesky factorisation
    kErrNonFinite = 4u,  // a p-sized draw became NaN or infinite
    kErrInput = 8u,      // invalid y or non-finite X at creation
};

// Layout of X in device memory: row-major, leading dimension ld elements,
// ld a multiple of 16 bytes, padding columns zero.
struct XLayout {
    const void* X;
    int xtype;   // 0 float32, 1 bfloat16
    uint32_t N;
    uint32_t p;
    uint32_t ld;
};

// ---- launchers (each enqueues on the given stream) --------------------------
struct ZPassArgs {
    XLayout x;
    const uint8_t* y;
    const float* beta32;
    Ctrl* ctrl;
    uint64_t seed;
    uint32_t chain;
    double* partial;   // grid rows x ld, per-block partial sums of X^T z
    float* zdbg;       // optional
    int32_t* adbg;     // optional
};
struct ZPassPlan {
    int blocks;    // grid size
    int rows_per_wave_tile;
    int chunks;
};
ZPassPlan zpass_plan(const XLayout& x, int num_cus);
hipError_t zpass_launch(const ZPassArgs& a, const ZPassPlan& plan, hipStream_t st);

// b[j] = sum over rows r < nrows of partial[r * ld + j], j < p, fixed order.
hipError_t reduce_cols_launch(const double* partial, int nrows, uint32_t ld, uint32_t p,
                              double* b, hipStream_t st);

// G = X^T X (p x p float64, leading dimension p); work must hold
// gram_work_doubles(x) doubles.
size_t gram_work_doubles(const XLayout& x, int num_cus);
hipError_t gram_launch(const XLayout& x, double* G, double* work, int num_cus, hipStream_t st);

// Input validation: sets kErrInput in ctrl if a y is not 0/1 or an X entry is
// not finite.
hipError_t validate_launch(const XLayout& x, const uint8_t* y, Ctrl* ctrl, hipStream_t st);

// Copy / convert a float32 N x p matrix (leading dimension p) into the padded
// library layout.
hipError_t pack_x_launch(const float* src, const XLayout& dst, hipStream_t st);

// p-side state on the device.
struct PState {
    uint32_t p;
    double* beta;      // p
    float* beta32;     // ld (padding zero)
    double* lam_m2;    // p
    double* nu_m1;     // p
    double* tau_m2;    // 1
    double* xi_m1;     // 1
    double* b;         // p: X^T z of the current sweep
    const double* G;   // p x p
    double* A;         // p x p workspace: Q, then the off-diagonal blocks of its
                       // upper Cholesky factor
    double* Ud;        // ceil(p/64) x 64 x 64: factors of the diagonal blocks
    double* vec;       // 4 p workspace (s / v / w / mu)
    Ctrl* ctrl;
    uint64_t seed;
    uint32_t chain;
    int small_lds_ok;  // the one-block LDS beta kernel fits (p <= 128)
};

// Whether the one-block beta kernel fits p on a device with max_lds bytes of
// LDS per block; pside_prepare raises that kernel's dynamic LDS limit.
bool beta_small_fits(uint32_t p, size_t max_lds);
hipError_t pside_prepare(size_t max_lds);

hipError_t lambda_launch(const PState& s, hipStream_t st);
hipError_t tau_launch(const PState& s, hipStream_t st);
hipError_t beta_launch(const PState& s, hipStream_t st);   // Q, Cholesky, solves, beta
hipError_t nuxi_launch(const PState& s, hipStream_t st);
hipError_t record_launch(const PState& s, double* ring_beta, double* ring_tau,
                         double* ring_lam, uint32_t thin, uint32_t capacity, hipStream_t st);
hipError_t advance_launch(Ctrl* ctrl, hipStream_t st);
hipError_t philox_test_launch(uint64_t seed, const uint32_t* ctr, uint32_t n, uint32_t* out,
                              hipStream_t st);

}  // namespace hsp
