// The p-side role of the sweep kernel: the conditionals of Eq. (12) other
// than z, in float64, computed by a group of gp blocks that run next to the
// z-pass blocks of the same launch.
//
//   lambda_j^-2 ~ Exp(nu_j^-1 + tau^-2 beta_j^2 / 2)
//   tau^-2      ~ Gamma((p+1)/2, rate xi^-1 + sum_j lambda_j^-2 beta_j^2 / 2)
//   nu_j^-1     ~ Exp(1 + lambda_j^-2),   xi^-1 ~ Exp(1 + tau^-2)
//   beta        ~ N(Q^-1 X^T z, Q^-1),  Q = X^T X + tau^-2 Lambda^-2
// (rate parameterisation, Eq. 11; tau^-2 is the Gamma draw of Section 5's
// sampling step, so tau^2 is inverse-gamma).  lambda, tau, nu, xi and the
// Cholesky factorisation of Q depend only on the previous sweep, so the group
// runs them while the z pass streams X; beta waits for the z pass.
//
// beta for p <= 16 (one block): Q packed in LDS, Q = U^T U by a right-looking
// Cholesky, then s ~ N(0, I), U v = s, U^T w = b, U mu = w, beta = mu + v
// (Section 5, beta steps ii-viii).
//
// beta for p > 16 (gp blocks, 64 x 64 tiles): a right-looking blocked
// Cholesky that applies the same row operations to an identity block, so it
// produces U and L^-1 = U^-T together (the factorisation of [Q | I]).  Then
//   y = L^-1 b + s,   beta = L^-T y = U^-1 U^-T b + U^-1 s,
// which is mean Q^-1 b plus noise with covariance U^-1 U^-T = Q^-1: the same
// draw as the substitutions, as two parallel triangular products that run
// after the z pass.
//
// Group barriers use a monotonic device counter; every wait is bounded in
// time and sets kErrTimeout instead of hanging.
#pragma once
#include <float.h>

#include "hsp_internal.hpp"
#include "philox.hpp"
#include "sync_dev.hpp"

namespace hsp {

// ---- bounded waits and group barriers ---------------------------------------------
struct Group {
    uint64_t* trace;           // this block's timestamp slots, or null
    Ctrl* ctrl;
    unsigned long long base;   // bar_count when this launch started
    unsigned long long zbase;  // z_count when this launch started
    uint32_t size;
    uint32_t n;                // barriers passed
    uint32_t slot;             // next trace slot
    uint32_t npotrf;           // diagonal tiles factored by this block
    uint64_t timeout;
};

// Block-uniform read of the failure flags that stop the group's work.
__device__ __forceinline__ bool group_failed(const Group& g, double* lds_flag) {
    __syncthreads();
    if (threadIdx.x == 0)
        lds_flag[0] = (__hip_atomic_load(&g.ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                       (kErrNotPD | kErrTimeout)) ? 1.0 : 0.0;
    __syncthreads();
    const bool f = lds_flag[0] != 0.0;
    __syncthreads();
    return f;
}

// Sleep about 64 * n cycles between polls.  Polls are coherent loads that
// bypass the L2 and all land on one memory channel: a tight loop from many
// blocks slows the z pass's stream, so every wait backs off exponentially.
__device__ __forceinline__ void backoff(uint32_t& n, uint32_t cap) {
    for (uint32_t i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(1);
    n = n < cap ? 2 * n : cap;
}

// Thread 0 only: wait until *ctr >= target, or give up after the timeout.
// Relaxed polls; what the caller reads afterwards it loads coherently.
__device__ __forceinline__ void wait_count(unsigned long long* ctr, unsigned long long target,
                                        Ctrl* ctrl, uint64_t timeout, uint32_t cap = 16) {
    const uint64_t t0 = wall_clock64();
    uint32_t nap = 1;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(&ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrTimeout)
            break;
        if (wall_clock64() - t0 > timeout) {
            atomicOr(&ctrl->err, kErrTimeout);
            break;
        }
        backoff(nap, cap);
    }
}

// Thread 0: next trace timestamp, or a given value (diagnostics only).
__device__ __forceinline__ void stamp(Group& g) {
    if (g.trace && threadIdx.x == 0 && g.slot + 1 < (uint32_t)kTraceSeq) g.trace[++g.slot] = wall_clock64();
}
__device__ __forceinline__ void stamp_value(Group& g, uint64_t v) {
    if (g.trace && threadIdx.x == 0 && g.slot + 1 < (uint32_t)kTraceSeq) g.trace[++g.slot] = v;
}

// Thread 0: timestamp into slot s of a diagonal-factorisation record (or none).
__device__ __forceinline__ void stamp_at(uint64_t* rec, int s) {
    if (rec && threadIdx.x == 0) rec[s] = wall_clock64();
}

// Thread 0 only: wait until *v[i] >= need[i] for i < n (the n loads of a poll
// are in flight together); false if the group is failing or the wait timed
// out.  The tiles read after a success are loaded coherently (ldc).
__device__ __forceinline__ bool wait_vers(uint32_t* const (&v)[3], const uint32_t (&need)[3], int n,
                                          Ctrl* ctrl, uint64_t timeout) {
    uint64_t t0 = 0;
    uint32_t nap = 1;
    for (int it = 0;; ++it) {
        uint32_t got[3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
            got[i] = i < n ? __hip_atomic_load(v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        bool ok = true;
#pragma unroll
        for (int i = 0; i < 3; ++i) ok = ok && (i >= n || got[i] >= need[i]);
        if (ok) return true;
        if (it == 0) t0 = wall_clock64();
        if (__hip_atomic_load(&ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
            (kErrTimeout | kErrNotPD))
            return false;
        if (wall_clock64() - t0 > timeout) {
            atomicOr(&ctrl->err, kErrTimeout);
            return false;
        }
        backoff(nap, 8);
    }
}

// Publish *ver = val (and *ver2 = val2) once this block's coherent tile
// stores are complete: every wave waits for its own stores first.
__device__ __forceinline__ void publish(uint32_t* ver, uint32_t val, uint32_t* ver2 = nullptr,
                                        uint32_t val2 = 0) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_store(ver, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ver2) __hip_atomic_store(ver2, val2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ void group_sync(Group& g) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&g.ctrl->bar_count, 1ull);
        if (g.size > 1)
            wait_count(&g.ctrl->bar_count, g.base + (unsigned long long)(g.n + 1) * g.size, g.ctrl,
                       g.timeout);
    }
    g.n++;
    stamp(g);
    __syncthreads();
}

// Block-wide float64 sum in a fixed order (identical result in every block).
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kThreads / kWave; ++w) s += red[w];
    __syncthreads();
    return s;
}

__device__ __forceinline__ uint32_t record_slot(Args& a, uint32_t k, bool* keep) {
    const uint32_t since = k - a.ctrl->draw_base;
    *keep = (a.mode & kModeRecord) && since % a.thin == 0;
    return *keep ? (since / a.thin - 1u) % a.capacity : 0u;
}

// ---- lambda^-2 and tau^-2 (every block of the group computes them) ---------------
// Returns tau^-2 (new if kModeTau).  Block `writer` stores lambda^-2 and tau^-2.
__device__ double hyper_lambda_tau(Args& a, uint32_t k, bool writer, double* red) {
    const uint32_t p = a.x.p;
    const double tau_old = *a.tau_m2;
    double acc = 0.0;
    uint32_t clamps = 0;
    bool bad = false;
    for (uint32_t j = threadIdx.x; j < p; j += kThreads) {
        const double bj = a.beta[j];
        double lam;
        if (a.mode & kModeLambda) {
            double rate = a.nu_m1[j] + tau_old * bj * bj / 2.0;
            if (!(rate >= DBL_MIN)) {
                rate = DBL_MIN;
                ++clamps;
            }
            const Words4 w = draw_words(a.seed, j, k, kTagLambda, 0, a.chain);
            lam = -log(u01d(w.w0)) / rate;
            if (!isfinite(lam)) bad = true;
            if (writer) stc(&a.lam_m2[j], lam);
        } else {
            lam = a.lam_m2[j];
        }
        acc += lam * bj * bj;
    }
    if (writer) {
        if (clamps) atomicAdd(&a.ctrl->clamps, (unsigned long long)clamps);
        if (bad) atomicOr(&a.ctrl->err, kErrNonFinite);
    }
    if (!(a.mode & kModeTau)) return tau_old;
    const double sum = block_sum(acc, red);
    // Cheng's GB: proposal m = 64 * round + lane, uniforms of Philox round m/2
    // (words 0-1 for even m, 2-3 for odd m); the lowest accepted m wins, which
    // is the first acceptance of the sequential algorithm.  (Section 5 uses 32
    // threads and a serial scan for the same purpose.)
    if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        const double rate = *a.xi_m1 + sum / 2.0;
        const double sh = ((double)p + 1.0) / 2.0;
        const double A = 1.0 / sqrt(2.0 * sh - 1.0);
        const double B = sh - log(4.0);
        const double C = sh + 1.0 / A;
        const double D = 1.0 + log(4.5);
        double g = __builtin_nan("");
        for (uint32_t round = 0; round < (1u << 16); ++round) {
            const uint32_t m = round * kWave + lane;
            const Words4 w = draw_words(a.seed, 0, k, kTagTau, m >> 1, a.chain);
            const double u1 = u01d((m & 1u) ? w.w2 : w.w0);
            const double u2 = u01d((m & 1u) ? w.w3 : w.w1);
            const double V = A * log(u1 / (1.0 - u1));
            const double X = sh * exp(V);
            const double Z = u1 * u1 * u2;
            const double R = B + C * V - X;
            const bool ok = (R + D - 4.5 * Z >= 0.0) || (R >= log(Z));
            const unsigned long long mask = __ballot(ok);
            if (mask) {
                g = __shfl(X, (int)(__ffsll((long long)mask) - 1));
                break;
            }
        }
        if (lane == 0) red[8] = g / rate;
    }
    __syncthreads();
    const double tau = red[8];
    // the other blocks may still be reading the old value: the new one goes to
    // a scratch slot and is published when the launch closes
    if (writer && threadIdx.x == 0) {
        stc(&a.vec[2 * p], tau);
        if (!isfinite(tau) || !(tau > 0.0)) atomicOr(&a.ctrl->err, kErrNonFinite);
    }
    __syncthreads();
    return tau;
}

// tau^-2 of this sweep: the scratch slot if it was drawn in this launch.
__device__ __forceinline__ double current_tau(Args& a) {
    // written by block 0 of the group in this launch: read past the scalar cache
    return (a.mode & kModeTau)
               ? __hip_atomic_load(a.vec + 2 * a.x.p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
               : *a.tau_m2;
}

// nu^-1 and xi^-1 from the (new) lambda^-2 and tau^-2 in memory.
__device__ void hyper_nu_xi(Args& a, uint32_t k) {
    const uint32_t p = a.x.p;
    for (uint32_t j = threadIdx.x; j < p; j += kThreads) {
        const Words4 w = draw_words(a.seed, j, k, kTagNu, 0, a.chain);
        a.nu_m1[j] = -log(u01d(w.w0)) / (1.0 + ldc(&a.lam_m2[j]));
    }
    if (threadIdx.x == 0) {
        const Words4 w = draw_words(a.seed, 0, k, kTagXi, 0, a.chain);
        *a.xi_m1 = -log(u01d(w.w0)) / (1.0 + current_tau(a));
    }
}

// ---- one-block path, p <= 16 -----------------------------------------------------
__device__ __forceinline__ uint32_t pk(uint32_t p, uint32_t i, uint32_t j) {
    // packed upper triangle, row-major: row i starts at i p - i (i - 1) / 2
    return i * p - (i * (i - 1u)) / 2u + (j - i);
}

__device__ double lane_elem(const double (&r)[2], uint32_t i) {
    const double v0 = __shfl(r[0], (int)(i & 63u));
    const double v1 = __shfl(r[1], (int)(i & 63u));
    return i < 64u ? v0 : v1;
}

// One wave: U^T x = r (forward) or U x = r (backward), U packed in LDS;
// lane l holds entries l and l + 64.
__device__ void wave_solve(const double* U, uint32_t p, double (&r)[2], bool forward) {
    const int lane = threadIdx.x & 63;
    if (forward) {
        for (uint32_t i = 0; i < p; ++i) {
            const double xi = lane_elem(r, i) / U[pk(p, i, i)];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t j = q * 64 + lane;
                if (j == i) r[q] = xi;
                else if (j > i && j < p) r[q] -= U[pk(p, i, j)] * xi;
            }
        }
    } else {
        for (int ii = (int)p - 1; ii >= 0; --ii) {
            const uint32_t i = (uint32_t)ii;
            const double xi = lane_elem(r, i) / U[pk(p, i, i)];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t j = q * 64 + lane;
                if (j == i) r[q] = xi;
                else if (j < i) r[q] -= U[pk(p, j, i)] * xi;
            }
        }
    }
}

// LDS offset (doubles) of b on the one-block path, past the packed factor.
constexpr uint32_t kSmallBOff = 512;
static_assert(kSmallP * (kSmallP + 1) / 2 <= (int)kSmallBOff && kSmallBOff + kSmallP <= (uint32_t)kLdsDoubles,
              "one-block path LDS layout");

__device__ void small_path(Args& a, Group& g, uint32_t k, double* lds) {
    const uint32_t p = a.x.p;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double tau = hyper_lambda_tau(a, k, true, lds);
    group_sync(g);  // lambda, tau in memory
    if (a.mode & kModeNuXi) hyper_nu_xi(a, k);
    bool bad = false;
    if (a.mode & kModeBeta) {
        double* U = lds;  // p (p + 1) / 2 doubles
        for (uint32_t i = ty; i < p; i += 16)
            for (uint32_t j = i + tx; j < p; j += 16)
                U[pk(p, i, j)] = a.G[(size_t)i * p + j] + (i == j ? tau * a.lam_m2[i] : 0.0);
        __syncthreads();
        // right-looking, row scaling deferred: step c subtracts
        // A[c][i] A[c][j] / A[c][c] from the trailing upper triangle
        for (uint32_t c = 0; c < p; ++c) {
            const double d = U[pk(p, c, c)];
            if (!(d > 0.0)) {
                bad = true;
                break;
            }
            const double inv = 1.0 / d;
            for (uint32_t i = c + 1 + ty; i < p; i += 16) {
                const double f = U[pk(p, c, i)] * inv;
                for (uint32_t j = i + tx; j < p; j += 16) U[pk(p, i, j)] -= f * U[pk(p, c, j)];
            }
            __syncthreads();
        }
        if (!bad) {
            for (uint32_t i = ty; i < p; i += 16) {
                const double rs = 1.0 / sqrt(U[pk(p, i, i)]);
                for (uint32_t j = i + 1 + tx; j < p; j += 16) U[pk(p, i, j)] *= rs;
            }
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < p; i += kThreads) U[pk(p, i, i)] = sqrt(U[pk(p, i, i)]);
            __syncthreads();
        } else if (threadIdx.x == 0) {
            atomicOr(&a.ctrl->err, kErrNotPD);
            for (uint32_t c = 0; c < p; ++c)
                if (!(U[pk(p, c, c)] > 0.0)) {
                    atomicCAS(&a.ctrl->chol_info, 0, (int)(c + 1));
                    break;
                }
        }
    }
    if (a.mode & (kModeZ | kModeBsum)) {
        if ((a.mode & kModeZ) && threadIdx.x == 0) {
            wait_count(&a.ctrl->z_count, g.zbase + a.zgroups, a.ctrl, a.timeout_ticks, 64);
        }
        __syncthreads();
        // b as the z groups (of this launch, or of an earlier multi-chain
        // pass) accumulated it, in the units of the stored X, unscaled
        // exactly; wave 0 takes it from LDS below
        for (uint32_t j = threadIdx.x; j < p; j += kThreads) {
            const double s = ldc(&a.bsum[j]) * a.xscale[j];
            a.b[j] = s;
            lds[kSmallBOff + j] = s;
        }
        __syncthreads();
    }
    bool keep;
    const uint32_t slot = record_slot(a, k, &keep);
    if ((a.mode & kModeBeta) && !bad && threadIdx.x < kWave) {
        const double* U = lds;
        const int lane = threadIdx.x;
        double v[2], w[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint32_t j = q * 64 + lane;
            v[q] = 0.0;
            w[q] = 0.0;
            if (j < p) {
                const Words4 wd = draw_words(a.seed, j, k, kTagBetaS, 0, a.chain);
                v[q] = box_muller_d(u01d(wd.w0), u01d(wd.w1));
                w[q] = (a.mode & (kModeZ | kModeBsum)) ? lds[kSmallBOff + j] : a.b[j];
            }
        }
        wave_solve(U, p, v, false);  // U v = s
        wave_solve(U, p, w, true);   // U^T w = b
        wave_solve(U, p, w, false);  // U mu = w
        bool nonfinite = false;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint32_t j = q * 64 + lane;
            if (j < p) {
                const double bj = w[q] + v[q];
                a.beta[j] = bj;
                a.beta32[j] = (float)(bj * a.xscale[j]);
                if (!isfinite(bj)) nonfinite = true;
                if (keep) a.ring_beta[(size_t)slot * p + j] = bj;
            }
        }
        if (__ballot(nonfinite) && lane == 0) atomicOr(&a.ctrl->err, kErrNonFinite);
    }
    if (keep) {
        __syncthreads();
        if (a.ring_lam)
            for (uint32_t j = threadIdx.x; j < p; j += kThreads) a.ring_lam[(size_t)slot * p + j] = ldc(&a.lam_m2[j]);
        if (threadIdx.x == 0) a.ring_tau[slot] = current_tau(a);
    }
}

// ---- tile path, p > 16 ----------------------------------------------------------
// The tile path works on P x P matrices, P = p rounded up to a multiple of 64,
// leading dimension P: Gp holds G with an identity block on the padding, so
// the factor, L^-1 and Q^-1 carry an identity block there too and no tile
// ever needs a bounds check.
typedef double Tile[kTile][kTileLd];

__device__ __forceinline__ uint32_t padded(uint32_t p) { return (p + kTile - 1) / kTile * kTile; }

// T[r][c] = M[(r0 + r) P + c0 + c] (+ tau * lam on the diagonal of Q when
// add_diag).  Thread t reads column t % 64 of rows t / 64 + 4q: every load
// instruction of a wave is one contiguous 512-byte row segment, and all 16
// loads of a thread are in flight together.
__device__ __forceinline__ void load_tile(Tile& T, const double* M, uint32_t P, uint32_t r0,
                                          uint32_t c0, bool add_diag, double tau,
                                          const double* lam, uint32_t p) {
    const int c = threadIdx.x & (kTile - 1), rb = threadIdx.x >> 6;
    const double* src = M + (size_t)(r0 + rb) * P + c0 + c;
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = ldc(src + (size_t)(4 * q) * P);
    if (add_diag) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const uint32_t gi = r0 + rb + 4 * q;
            if (gi == c0 + c && gi < p) v[q] += tau * ldc(lam + gi);
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) T[rb + 4 * q][c] = v[q];
}

// load_tile for two tiles with every global load issued before any LDS store.
__device__ __forceinline__ void load_tiles(Tile& S, const double* MS, uint32_t rs, uint32_t cs,
                                           Tile& T, const double* MT, uint32_t rt, uint32_t ct,
                                           uint32_t P) {
    const int c = threadIdx.x & (kTile - 1), rb = threadIdx.x >> 6;
    const double* s0 = MS + (size_t)(rs + rb) * P + cs + c;
    const double* t0 = MT + (size_t)(rt + rb) * P + ct + c;
    double v[16], w[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        v[q] = ldc(s0 + (size_t)(4 * q) * P);
        w[q] = ldc(t0 + (size_t)(4 * q) * P);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        S[rb + 4 * q][c] = v[q];
        T[rb + 4 * q][c] = w[q];
    }
}

// ---- 64 x 64 x 64 tile products on the FP64 matrix cores ----------------------
// v_mfma_f64_16x16x4f64 computes D(16x16) += A(16x4) B(4x16); lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[l / 16 + 4 r][l % 16]
// in its r-th result.  Wave w owns the 32 x 32 quadrant at rows 32 (w / 2),
// columns 32 (w % 2) as 2 x 2 blocks of 16 x 16; per k-step of 4 it reads
// four 64-lane fragments from LDS for four matrix operations.
typedef double Acc4 __attribute__((ext_vector_type(4)));
struct MAcc {
    Acc4 v[2][2];
};

// acc = S^T T, or S T when TA (S read transposed: its rows are the product's rows).
template <bool TA = false>
__device__ __forceinline__ void gemm_tn(const Tile& S, const Tile& T, MAcc& acc) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i0 = 32 * (wave >> 1), j0 = 32 * (wave & 1);
    const int kr = lane >> 4, cc = lane & 15;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc.v[bi][bj] = Acc4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int q0 = 0; q0 < kTile; q0 += 4) {
        const double a0 = TA ? S[i0 + cc][q0 + kr] : S[q0 + kr][i0 + cc];
        const double a1 = TA ? S[i0 + 16 + cc][q0 + kr] : S[q0 + kr][i0 + 16 + cc];
        const double b0 = T[q0 + kr][j0 + cc], b1 = T[q0 + kr][j0 + 16 + cc];
        acc.v[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.v[0][0], 0, 0, 0);
        acc.v[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.v[0][1], 0, 0, 0);
        acc.v[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.v[1][0], 0, 0, 0);
        acc.v[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc.v[1][1], 0, 0, 0);
    }
}

// The matrix-core layout of a 64 x 64 tile at (r0, c0) of M: lane l of wave w
// holds rows r0 + 32 (w / 2) + 16 bi + l / 16 + 4 r, column c0 + 32 (w % 2) +
// 16 bj + l % 16; each group of 16 lanes covers a 128-byte row segment.
struct MTile {
    double v[2][2][4];
};

// Load a tile in that layout (zeros for a null M), with tau * lam added on
// Q's diagonal when add_diag.  Issued before a product, the loads overlap it.
__device__ __forceinline__ void load_tile_m(MTile& o, const double* M, uint32_t P, uint32_t r0,
                                            uint32_t c0, bool add_diag, double tau, const double* lam,
                                            uint32_t p) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t ri = r0 + 32 * (wave >> 1) + (lane >> 4);
    const uint32_t cj = c0 + 32 * (wave & 1) + (lane & 15);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                o.v[bi][bj][r] = M ? ldc(M + (size_t)(ri + 16 * bi + 4 * r) * P + cj + 16 * bj) : 0.0;
    if (add_diag) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint32_t gi = ri + 16 * bi + 4 * r, gj = cj + 16 * bj;
                    if (gi == gj && gi < p) o.v[bi][bj][r] += tau * ldc(lam + gi);
                }
    }
}

// M(r0.., c0..) = old + sign * acc, sixteen stores back to back.
__device__ __forceinline__ void put_tile_m(double* M, uint32_t P, uint32_t r0, uint32_t c0,
                                           const MAcc& acc, double sign, const MTile& old) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t ri = r0 + 32 * (wave >> 1) + (lane >> 4);
    const uint32_t cj = c0 + 32 * (wave & 1) + (lane & 15);
    double out[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[bi][bj][r] = fma(sign, acc.v[bi][bj][r], old.v[bi][bj][r]);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) stc(M + (size_t)(ri + 16 * bi + 4 * r) * P + cj + 16 * bj, out[bi][bj][r]);
}

// X = old + sign * acc in LDS (the matrix-core layout, X's own rows and columns).
__device__ __forceinline__ void acc_to_lds(Tile& X, const MAcc& acc, double sign, const MTile& old) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ri = 32 * (wave >> 1) + (lane >> 4), cj = 32 * (wave & 1) + (lane & 15);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                X[ri + 16 * bi + 4 * r][cj + 16 * bj] = fma(sign, acc.v[bi][bj][r], old.v[bi][bj][r]);
}

__device__ __forceinline__ double rdlane(double v, int l) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1 / sqrt(d) for d > 0: the hardware estimate and one Newton step.
__device__ __forceinline__ double rsqrt_nr(double d) {
    const double y = __builtin_amdgcn_rsq(d);
    const double e = fma(-d * y, y, 1.0);  // 1 - d y^2
    return fma(0.5 * y, e, y);
}

// Factor a 64 x 64 diagonal block: S holds its upper part (zeros below,
// identity beyond the matrix edge); on return S = U (upper) and T = U^-T
// (lower), i.e. the factorisation of [S | I] by row operations.
//
// Four row panels of 16.  For each, wave 0 eliminates the panel in registers,
// columns across the lanes.  At step c the pivot d is lane (r0 + c)'s entry of
// row c and every later panel row i loses m_i / d times row c, m_i being row
// c's entry in lane r0 + i, in the S part and in the identity part alike; row
// c is then scaled by 1/sqrt(d).  The multipliers are read from row c before
// it is scaled, so those reads do not wait for the square root, and row c + 1
// is updated first, so the next pivot's chain overlaps the other rows'
// updates.  That factors the panel's diagonal block and solves its other
// columns at once.  Then all four waves subtract the panel's rank-16
// contribution from the rows below on the matrix cores, as 16 x 16 blocks:
// S(I, J) -= U(P, I)^T U(P, J) for P < I <= J, and T(I, J) -= U(P, I)^T T(P, J)
// for J <= P < I.  Returns false on a non-positive pivot (uniformly: the flag
// goes through LDS).
__device__ bool factor_diag(Tile& S, Tile& T, uint64_t* rec) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* flag = &T[kTile - 1][kTile];  // padding corner, not part of the tile
    // T starts as the identity: wave 0 makes its first panel's rows in
    // registers, the other waves write rows 16.. meanwhile (the first
    // barrier below orders them before any reader).
    if (wave > 0)
        for (int e = threadIdx.x - kWave + 16 * kTile; e < kTile * kTile; e += kThreads - kWave)
            T[e / kTile][e % kTile] = e / kTile == e % kTile ? 1.0 : 0.0;
#pragma unroll
    for (int P = 0; P < 4; ++P) {
        const int r0 = 16 * P;
        if (wave == 0) {
            double a[16], w[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                a[c] = S[r0 + c][lane];
                w[c] = P == 0 ? (lane == c ? 1.0 : 0.0) : T[r0 + c][lane];
            }
            bool ok = true;
            double d = rdlane(a[0], r0);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                double m[16];
#pragma unroll
                for (int i = c + 1; i < 16; ++i) m[i] = rdlane(a[c], r0 + i);
                ok = ok && (d > 0.0);
                const double rs = rsqrt_nr(d);
                const double inv = rs * rs;
                const double ta = a[c] * inv, tw = w[c] * inv;
                double dn = 0.0;
                if (c + 1 < 16) {
                    a[c + 1] = fma(-m[c + 1], ta, a[c + 1]);
                    w[c + 1] = fma(-m[c + 1], tw, w[c + 1]);
                    dn = rdlane(a[c + 1], r0 + c + 1);
                }
#pragma unroll
                for (int i = c + 2; i < 16; ++i) {
                    a[i] = fma(-m[i], ta, a[i]);
                    w[i] = fma(-m[i], tw, w[i]);
                }
                a[c] = lane == r0 + c ? d * rs : a[c] * rs;
                w[c] *= rs;
                d = dn;
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                S[r0 + c][lane] = lane >= r0 + c ? a[c] : 0.0;
                T[r0 + c][lane] = w[c];
            }
            if (lane == 0) *flag = ok ? 0.0 : 1.0;
        }
        __syncthreads();
        stamp_at(rec, 1 + 2 * P);
        if (*flag != 0.0) return false;
        if (P < 3) {
            // blocks below the panel: S part (I, J), P < I <= J <= 3, then the
            // T part (I, J), I > P, J <= P; wave w takes blocks w, w + 4, ...
            const int nS = (3 - P) * (4 - P) / 2, nT = (3 - P) * (P + 1);
            const int kr = lane >> 4, cc = lane & 15;
            for (int blk = wave; blk < nS + nT; blk += kThreads / kWave) {
                int I, J;
                bool spart = blk < nS;
                if (spart) {
                    int idx = blk;
                    I = P + 1;
                    while (idx >= 4 - I) {
                        idx -= 4 - I;
                        ++I;
                    }
                    J = I + idx;
                } else {
                    const int t2 = blk - nS;
                    I = P + 1 + t2 / (P + 1);
                    J = t2 % (P + 1);
                }
                Tile& B = spart ? S : T;
                Acc4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const double x = S[r0 + 4 * kk + kr][16 * I + cc];
                    const double y = B[r0 + 4 * kk + kr][16 * J + cc];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) B[16 * I + kr + 4 * r][16 * J + cc] -= acc[r];
            }
        }
        __syncthreads();
        stamp_at(rec, 2 + 2 * P);
    }
    stamp_at(rec, 9);
    return true;
}

// Factor diagonal block kb held in S (its upper part; the rest is not read)
// and store L^-1_kk = U_kk^-T into Linv: the triangular solves read it from
// there (U_kk itself is needed by nothing after this block).  Reports a
// failed pivot.  On return S = U_kk and T = U_kk^-T.
__device__ void diag_factor(Args& a, uint32_t kb, Tile& S, Tile& T, uint64_t* rec) {
    const uint32_t P = padded(a.x.p), k0 = kb * kTile;
    stamp_at(rec, 0);
    if (factor_diag(S, T, rec)) {
        const int c = threadIdx.x & (kTile - 1), rb = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = rb + 4 * q;
            stc(a.Linv + (size_t)(k0 + r) * P + k0 + c, T[r][c]);
        }
    } else if (threadIdx.x == 0) {
        atomicOr(&a.ctrl->err, kErrNotPD);
        atomicCAS(&a.ctrl->chol_info, 0, (int)(k0 + 1));
    }
    __syncthreads();
    stamp_at(rec, 10);
}

// Run block `rank`'s list of factorisation tasks.  Tile versions: U tile
// (i, j), i <= j, has had v of its i updates (plus 1 once final); L^-1 tile
// (i, j), j <= i, v of its i - j updates (plus 1 once final).  Each task waits
// for the versions it reads, then publishes the version it wrote.  Returns
// false if the group is failing.
__device__ bool run_tasks(Args& a, Group& g, uint32_t rank, double tau, Tile& S, Tile& T,
                          double* flag) {
    const uint32_t p = a.x.p, P = padded(p), nt = P / kTile;
    uint32_t* vU = a.ver;
    uint32_t* vL = a.ver + nt * nt;
    // Block 0 (or a group of one) runs its own list; the others claim tasks
    // from the shared queue in order, each reserving its next task when it
    // starts one.  The claimed index travels to the block through LDS.
    const bool queue = g.size > 1 && rank > 0;
    const uint32_t n0 = queue ? a.task_off[1] : 0u, n1 = queue ? a.task_off[2] : a.task_off[1];
    double* next_lds = &T[kTile - 2][kTile];  // padding, not part of the tile
    uint32_t n = n0;
    if (queue) {
        if (threadIdx.x == 0) *next_lds = (double)atomicAdd(&a.ctrl->task_next, 1u);
        __syncthreads();
        n = n0 + (uint32_t)*next_lds;
        __syncthreads();
    }
    while (n < n1) {
        const uint32_t code = a.tasks[n];
        const uint32_t type = code & 3u, part = (code >> 2) & 1u, kb = (code >> 3) & kTaskField,
                       ib = (code >> 11) & kTaskField, jb = (code >> 19) & kTaskField;
        uint32_t reserved = 0;
        if (threadIdx.x == 0) {
            if (queue) reserved = atomicAdd(&a.ctrl->task_next, 1u);
            uint32_t* v[3] = {nullptr, nullptr, nullptr};
            uint32_t need[3] = {0u, 0u, 0u};
            int nv;
            if (type == kTaskPotrf) {
                v[0] = &vU[kb * nt + kb], need[0] = kb;
                nv = 1;
            } else if (type == kTaskPanel) {
                v[0] = &vU[(kb - 1) * nt + kb], need[0] = kb - 1;
                v[1] = &vU[kb * nt + kb], need[1] = kb - 1;
                nv = 2;
            } else if (type == kTaskTrsm) {
                v[0] = &vU[kb * nt + kb], need[0] = kb + 1;
                if (part == 0) v[1] = &vU[kb * nt + jb], need[1] = kb;
                else v[1] = &vL[kb * nt + jb], need[1] = kb - jb;
                nv = 2;
            } else {
                v[0] = &vU[kb * nt + ib], need[0] = kb + 1;
                if (part == 0) {
                    v[1] = &vU[kb * nt + jb], need[1] = kb + 1;
                    v[2] = &vU[ib * nt + jb], need[2] = kb;
                } else {
                    v[1] = &vL[kb * nt + jb], need[1] = kb - jb + 1;
                    v[2] = &vL[ib * nt + jb], need[2] = kb - jb;
                }
                nv = 3;
            }
            const bool w = wait_vers(v, need, nv, a.ctrl, g.timeout);
            *flag = w ? 0.0 : 1.0;
        }
        __syncthreads();
        stamp_value(g, n + 1u);
        stamp(g);
        if (*flag != 0.0) return false;
        const uint32_t k0 = kb * kTile;
        uint32_t* out = nullptr;   // version published when the task is done
        uint32_t* out2 = nullptr;  // a diagonal L^-1 tile, final at version 1
        uint32_t val = 0;
        if (type == kTaskPotrf || type == kTaskPanel) {
            uint64_t* rec = nullptr;
            if (g.trace && g.npotrf < (uint32_t)kTraceRecs) rec = g.trace + kTraceSeq + kTraceRec * g.npotrf;
            g.npotrf++;
            if (type == kTaskPotrf) {
                load_tile(S, kb == 0 ? a.Gp : a.A, P, k0, k0, kb == 0, tau, a.lam_m2, p);
                __syncthreads();
                stamp(g);
            } else {
                // U_{k-1,k} = D_{k-1}^T A_{k-1,k} with D_{k-1}^T still in T, then
                // A_kk -= U_{k-1,k}^T U_{k-1,k}, all in this block
                const uint32_t km = kb - 1, r1 = km * kTile;
                const double* src = km == 0 ? a.Gp : a.A;
                MTile dg;
                load_tile_m(dg, src, P, k0, k0, km == 0, tau, a.lam_m2, p);
                load_tile(S, src, P, r1, k0, false, 0.0, nullptr, p);
                __syncthreads();
                stamp(g);
                MAcc acc;
                gemm_tn<true>(T, S, acc);
                MTile zero;
                load_tile_m(zero, nullptr, P, 0, 0, false, 0.0, nullptr, p);
                put_tile_m(a.A, P, r1, k0, acc, 1.0, zero);
                __syncthreads();
                acc_to_lds(S, acc, 1.0, zero);
                __syncthreads();
                gemm_tn(S, S, acc);
                // U_{k-1,k} is published once its stores are complete; the
                // product above hid their latency
                publish(&vU[km * nt + kb], kb);
                acc_to_lds(S, acc, -1.0, dg);
                __syncthreads();
            }
            diag_factor(a, kb, S, T, rec);
            if (threadIdx.x == 0 &&
                (__hip_atomic_load(&a.ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrNotPD))
                *flag = 1.0;
            __syncthreads();
            if (*flag != 0.0) return false;
            out = &vU[kb * nt + kb];
            val = kb + 1;
            out2 = &vL[kb * nt + kb];
        } else if (type == kTaskTrsm) {
            // row kb times U_kk^-1: X_kj = L^-1_kk X_kj, L^-1_kk from Linv
            const uint32_t j0 = jb * kTile;
            load_tiles(S, a.Linv, k0, k0, T, part == 0 ? (kb == 0 ? a.Gp : a.A) : a.Linv, k0, j0, P);
            __syncthreads();
            stamp(g);
            MAcc acc;
            gemm_tn<true>(S, T, acc);
            MTile zero;
            load_tile_m(zero, nullptr, P, 0, 0, false, 0.0, nullptr, p);
            put_tile_m(part == 0 ? a.A : a.Linv, P, k0, j0, acc, 1.0, zero);
            out = part == 0 ? &vU[kb * nt + jb] : &vL[kb * nt + jb];
            val = part == 0 ? kb + 1 : kb - jb + 1;
        } else {
            // A_ij -= U_ki^T U_kj  or  L^-1_ij -= U_ki^T L^-1_kj; the three
            // tiles' loads are in flight together
            MTile old;
            if (part == 0)
                load_tile_m(old, kb == 0 ? a.Gp : a.A, P, ib * kTile, jb * kTile, kb == 0 && ib == jb, tau,
                            a.lam_m2, p);
            else
                load_tile_m(old, jb == kb ? nullptr : a.Linv, P, ib * kTile, jb * kTile, false, 0.0, nullptr, p);
            load_tiles(S, a.A, k0, ib * kTile, T, part == 0 ? a.A : a.Linv, k0, jb * kTile, P);
            __syncthreads();
            stamp(g);
            MAcc acc;
            gemm_tn(S, T, acc);
            put_tile_m(part == 0 ? a.A : a.Linv, P, ib * kTile, jb * kTile, acc, -1.0, old);
            out = part == 0 ? &vU[ib * nt + jb] : &vL[ib * nt + jb];
            val = part == 0 ? kb + 1 : kb - jb + 1;
        }
        if (threadIdx.x == 0 && queue) *next_lds = (double)reserved;
        publish(out, val, out2, 1u);
        stamp(g);
        n = queue ? n0 + (uint32_t)*next_lds : n + 1;
        __syncthreads();
    }
    return true;
}

// beta = U^-1 (U^-T b + s) by blocked substitution (p > kSubstP: there the
// factorisation leaves L^-1 out beyond its diagonal tiles, half of its flops).
// Block r of the group owns tile rows r, r + gp, ...  Forward, its rows in
// increasing order: the owner of row i subtracts U_ki^T w_k from b_i for each
// k < i as soon as row k's flag is up, then w_i = L^-1_ii r_i (the diagonal
// tile of L^-1 the factorisation stored), stores it and raises row i's flag.
// Backward, its rows in decreasing order: r_i = w_i + s_i - sum_{k > i}
// U_ik beta_k, beta_i = U_ii^-1 r_i = (L^-1_ii)^T r_i.  A row waits only on
// rows finished before it in the same direction, so the solve cannot
// deadlock.  Flags sit after the tile versions and are cleared with them.
__device__ void subst_solve(Args& a, Group& g, uint32_t rank, uint32_t k, double* lds, bool from_sum) {
    const uint32_t p = a.x.p, P = padded(p), nt = P / kTile;
    uint32_t* ff = a.ver + 2 * nt * nt;  // forward: w_i stored
    uint32_t* fb = ff + nt;              // backward: beta_i stored
    double* yv = a.vec;                  // w (then read back for y = w + s)
    const double* s_noise = a.vec + p;
    double* rv = lds;                    // the owned row's running vector (64)
    double* part = lds + kTile;          // 4 x 64 partial sums
    double* flag = lds + 5 * kTile;
    const int c = threadIdx.x & (kTile - 1), q = threadIdx.x >> 6;
    auto b_at = [&](uint32_t j) -> double {
        if (j >= p) return 0.0;
        return from_sum ? ldc(&a.bsum[j]) * a.xscale[j] : a.b[j];
    };
    auto wait_row = [&](uint32_t* f) -> bool {
        if (threadIdx.x == 0) {
            uint32_t* v[3] = {f, nullptr, nullptr};
            const uint32_t need[3] = {1u, 0u, 0u};
            *flag = wait_vers(v, need, 1, a.ctrl, g.timeout) ? 0.0 : 1.0;
        }
        __syncthreads();
        return *flag == 0.0;
    };
    // rv -= the four partial sums (then every thread sees the new rv)
    auto fold = [&](double acc) {
        part[q * kTile + c] = acc;
        __syncthreads();
        if (threadIdx.x < (uint32_t)kTile)
            rv[c] -= (part[c] + part[kTile + c]) + (part[2 * kTile + c] + part[3 * kTile + c]);
        __syncthreads();
    };
    bool ok = true;
    for (uint32_t i = rank; ok && i < nt; i += g.size) {
        const uint32_t i0 = i * kTile;
        if (threadIdx.x < (uint32_t)kTile) rv[c] = b_at(i0 + c);
        __syncthreads();
        for (uint32_t kk = 0; ok && kk < i; ++kk) {
            if (!(ok = wait_row(&ff[kk]))) break;
            // (U_kk,i^T w_kk)_c: thread (q, c) sums rows q, q + 4, ... of the tile
            double acc = 0.0;
#pragma unroll 4
            for (int j = 0; j < 16; ++j) {
                const uint32_t row = kk * kTile + q + 4 * j;
                const double wv = row < p ? ldc(&yv[row]) : 0.0;
                acc = fma(ldc(&a.A[(size_t)row * P + i0 + c]), wv, acc);
            }
            fold(acc);
        }
        if (!ok) break;
        // w_i = L^-1_ii r: thread (q, c) takes row c's columns 16 q .. 16 q + 15
        double acc = 0.0;
#pragma unroll 4
        for (int j = 0; j < 16; ++j)
            acc = fma(ldc(&a.Linv[(size_t)(i0 + c) * P + i0 + 16 * q + j]), rv[16 * q + j], acc);
        part[q * kTile + c] = acc;
        __syncthreads();
        if (threadIdx.x < (uint32_t)kTile && i0 + c < p)
            stc(&yv[i0 + c], (part[c] + part[kTile + c]) + (part[2 * kTile + c] + part[3 * kTile + c]));
        publish(&ff[i], 1u);
    }
    bool keep;
    const uint32_t slot = record_slot(a, k, &keep);
    bool nonfinite = false;
    const uint32_t nown = rank < nt ? (nt - 1 - rank) / g.size + 1 : 0u;
    for (uint32_t o = nown; ok && o-- > 0;) {
        const uint32_t i = rank + o * g.size, i0 = i * kTile;
        if (threadIdx.x < (uint32_t)kTile) rv[c] = i0 + c < p ? ldc(&yv[i0 + c]) + ldc(&s_noise[i0 + c]) : 0.0;
        __syncthreads();
        for (uint32_t kk = nt - 1; ok && kk > i; --kk) {
            if (!(ok = wait_row(&fb[kk]))) break;
            // (U_i,kk beta_kk)_c: thread (q, c) takes row c's columns 16 q .. 16 q + 15
            double acc = 0.0;
#pragma unroll 4
            for (int j = 0; j < 16; ++j) {
                const uint32_t col = kk * kTile + 16 * q + j;
                const double bv = col < p ? ldc(&a.beta[col]) : 0.0;
                acc = fma(ldc(&a.A[(size_t)(i0 + c) * P + col]), bv, acc);
            }
            fold(acc);
        }
        if (!ok) break;
        // beta_i = (L^-1_ii)^T r: thread (q, c) sums rows q, q + 4, ... of column c
        double acc = 0.0;
#pragma unroll 4
        for (int j = 0; j < 16; ++j) {
            const uint32_t r = q + 4 * j;
            acc = fma(ldc(&a.Linv[(size_t)(i0 + r) * P + i0 + c]), rv[r], acc);
        }
        part[q * kTile + c] = acc;
        __syncthreads();
        if (threadIdx.x < (uint32_t)kTile && i0 + c < p) {
            const uint32_t col = i0 + c;
            const double bi = (part[c] + part[kTile + c]) + (part[2 * kTile + c] + part[3 * kTile + c]);
            stc(&a.beta[col], bi);
            a.beta32[col] = (float)(bi * a.xscale[col]);
            if (!isfinite(bi)) nonfinite = true;
            if (keep) {
                a.ring_beta[(size_t)slot * p + col] = bi;
                if (a.ring_lam) a.ring_lam[(size_t)slot * p + col] = ldc(&a.lam_m2[col]);
            }
        }
        publish(&fb[i], 1u);
    }
    if (nonfinite) atomicOr(&a.ctrl->err, kErrNonFinite);
    if (keep && rank == 0 && threadIdx.x == 0) a.ring_tau[slot] = current_tau(a);
    // no block leaves before every flag it may wait on is up: the launch's
    // closing block clears them after this barrier
    group_sync(g);
}

__device__ void tile_path(Args& a, Group& g, uint32_t rank, uint32_t k, double* lds) {
    const uint32_t p = a.x.p, P = padded(p);
    Tile& S = *reinterpret_cast<Tile*>(lds);
    Tile& T = *reinterpret_cast<Tile*>(lds + kTile * kTileLd);
    double* flag = lds + 2 * kTile * kTileLd - 1;  // T's unused padding corner
    double* s_noise = a.vec + p;
    bool ok = true;
    if (!(a.mode & kModePost)) {
        const double tau = hyper_lambda_tau(a, k, rank == 0, lds);
        group_sync(g);  // lambda^-2 and the new tau^-2 in memory
        if (rank == g.size - 1) {
            if (a.mode & kModeNuXi) hyper_nu_xi(a, k);
            if (a.mode & kModeBeta)
                for (uint32_t i = threadIdx.x; i < p; i += kThreads) {
                    const Words4 w = draw_words(a.seed, i, k, kTagBetaS, 0, a.chain);
                    stc(&s_noise[i], box_muller_d(u01d(w.w0), u01d(w.w1)));
                }
        }
        if (a.mode & kModeBeta) {
            // Factorisation of [Q | I]: U in A (upper), L^-1 = U^-T in Linv
            // (lower), as this block's list of tile tasks.
            ok = run_tasks(a, g, rank, tau, S, T, flag);
            group_sync(g);
            ok = ok && !group_failed(g, flag);
        }
    } else {
        // an earlier launch of this sweep drew lambda, tau, nu, xi and the
        // noise of beta and factored Q; its failure flags are in memory
        ok = !group_failed(g, flag);
    }
    if (a.mode & kModePre) return;  // b is taken by a later launch of this sweep

    if (a.mode & kModeZ) {
        if (threadIdx.x == 0) {
            wait_count(&a.ctrl->z_count, g.zbase + a.zgroups, a.ctrl, a.timeout_ticks, 64);
        }
        if (g.trace && threadIdx.x == 0) g.trace[kTraceSlots - 1] = wall_clock64();
        __syncthreads();
    }
    // b = X^T z into LDS (zero on the padding), as the z groups accumulated
    // it; block 0 also stores it.  A vector too long for the LDS (big) is
    // read from memory where it is used instead.
    const bool big = P + 16 * 17 > (uint32_t)kLdsDoubles;
    const bool from_sum = (a.mode & (kModeZ | kModeBsum)) != 0;
    auto b_at = [&](uint32_t j) -> double {
        if (j >= p) return 0.0;
        return from_sum ? ldc(&a.bsum[j]) * a.xscale[j] : a.b[j];  // unscaled exactly
    };
    double* bl = lds;
    for (uint32_t j = threadIdx.x; j < P; j += kThreads) {
        const double s = b_at(j);
        if (from_sum && rank == 0 && j < p) a.b[j] = s;
        if (!big) bl[j] = s;
    }
    __syncthreads();

    if ((a.mode & kModeBeta) && ok && a.subst) {
        subst_solve(a, g, rank, k, lds, from_sum);
    } else if ((a.mode & kModeBeta) && ok) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        // y = L^-1 b + s, four rows per wave at a time.  L^-1 is zero above the
        // diagonal and the identity on the padding, and b is zero there, so
        // the sums need no bounds: row i runs over every column up to the
        // group's last row.  Rows are dealt so that each wave gets short and
        // long ones.
        double* yv = a.vec;
        for (uint32_t i0 = (rank * 4 + wave) * 4; i0 < p; i0 += g.size * 16) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            const double* L0 = a.Linv + (size_t)i0 * P;
            const uint32_t jn = i0 + 4;
            uint32_t j = lane;
            for (; j + 192 < jn; j += 256) {
                double x[4][4], bj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    bj[u] = big ? b_at(j + 64 * u) : bl[j + 64 * u];
#pragma unroll
                    for (int r = 0; r < 4; ++r) x[u][r] = ldc(L0 + (size_t)r * P + j + 64 * u);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[r] = fma(x[u][r], bj[u], acc[r]);
            }
            for (; j < jn; j += 64) {
                const double bj = big ? b_at(j) : bl[j];
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = fma(ldc(L0 + (size_t)r * P + j), bj, acc[r]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) acc[r] += __shfl_xor(acc[r], off);
            if (lane < 4 && i0 + lane < p) {
                double yi = acc[0];
#pragma unroll
                for (int r = 1; r < 4; ++r) yi = lane == r ? acc[r] : yi;
                stc(&yv[i0 + lane], yi + ldc(&s_noise[i0 + lane]));
            }
        }
        group_sync(g);
        // beta = L^-T y, y from LDS (zero on the padding); column j sums rows
        // i >= j, the rest of L^-1 being zero.  Block r takes two 16-column
        // blocks, one from each end (columns 16 r and P - 16 (r + 1) on), so
        // every block reads about the same number of rows; 16 row groups per
        // column, four rows of loads in flight each.
        double* yl = lds;
        if (!big)
            for (uint32_t j = threadIdx.x; j < P; j += kThreads) yl[j] = j < p ? ldc(&yv[j]) : 0.0;
        auto y_at = [&](uint32_t i) -> double { return big ? (i < p ? ldc(&yv[i]) : 0.0) : yl[i]; };
        double* red = big ? lds : lds + P;
        __syncthreads();
        bool keep;
        const uint32_t slot = record_slot(a, k, &keep);
        const int tc = threadIdx.x & 15, tr = threadIdx.x >> 4;
        bool nonfinite = false;
        for (uint32_t cb0 = rank * 16; cb0 < P / 2; cb0 += g.size * 16) {
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const uint32_t cb = half == 0 ? cb0 : P - 16 - cb0;
                const uint32_t col = cb + tc;
                const double* Lc = a.Linv + col;
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                uint32_t i = cb + tr;
                // sixteen loads in flight; the same accumulation order as
                // the four-row loop below
                for (; i + 240 < P; i += 256) {
                    double x[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) x[u] = ldc(Lc + (size_t)(i + 16 * u) * P);
#pragma unroll
                    for (int u = 0; u < 16; ++u) acc[u & 3] = fma(x[u], y_at(i + 16 * u), acc[u & 3]);
                }
                for (; i + 48 < P; i += 64)
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[u] = fma(ldc(Lc + (size_t)(i + 16 * u) * P), y_at(i + 16 * u), acc[u]);
                for (; i < P; i += 16) acc[0] = fma(ldc(Lc + (size_t)i * P), y_at(i), acc[0]);
                red[tr * 17 + tc] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
                __syncthreads();
                if (tr == 0 && col < p) {
                    double bi = 0.0;
                    for (int q = 0; q < 16; ++q) bi += red[q * 17 + tc];
                    a.beta[col] = bi;
                    a.beta32[col] = (float)(bi * a.xscale[col]);
                    if (!isfinite(bi)) nonfinite = true;
                    if (keep) {
                        a.ring_beta[(size_t)slot * p + col] = bi;
                        if (a.ring_lam) a.ring_lam[(size_t)slot * p + col] = ldc(&a.lam_m2[col]);
                    }
                }
                __syncthreads();
            }
        }
        if (nonfinite) atomicOr(&a.ctrl->err, kErrNonFinite);
        if (keep && rank == 0 && threadIdx.x == 0) a.ring_tau[slot] = current_tau(a);
    }
}

// The whole p-side role of block `rank` of the group.
__device__ __forceinline__ void pside_role(Args& a, uint32_t rank, uint32_t k, double* lds) {
    Group g;
    g.trace = a.trace ? a.trace + (size_t)rank * kTraceSlots : nullptr;
    if (g.trace && threadIdx.x == 0) g.trace[0] = wall_clock64();
    g.ctrl = a.ctrl;
    g.base = a.ctrl->bar_epoch;
    g.zbase = a.ctrl->z_epoch;
    g.size = a.gp;
    g.n = 0;
    g.slot = 0;
    g.npotrf = 0;
    g.timeout = a.timeout_ticks;
    // the two-launch split is for the tile path; a launch never asks the
    // one-block path for half a sweep
    if (a.x.p <= (uint32_t)kSmallP) {
        if (!(a.mode & (kModePre | kModePost))) small_path(a, g, k, lds);
    } else {
        tile_path(a, g, rank, k, lds);
    }
    // the last barrier above was passed by every block of the group, and the
    // z-pass blocks have all finished if they ran: close the launch
    if (rank == 0) {
        __syncthreads();
        if (threadIdx.x == 0) {
            a.ctrl->bar_epoch = g.base + (unsigned long long)g.n * g.size;
            if (a.mode & kModeZ) a.ctrl->z_epoch = g.zbase + a.zgroups;
            if (a.mode & kModeTau) *a.tau_m2 = current_tau(a);
            if (a.mode & kModeAdvance) a.ctrl->sweep = k;
        }
        if (a.x.p > (uint32_t)kSmallP && (a.mode & kModeBeta) && !(a.mode & kModePost)) {
            const uint32_t nt = padded(a.x.p) / kTile;
            // tile versions, and the substitution's row flags after them
            const uint32_t nver = 2 * nt * nt + (a.subst ? 2 * nt : 0u);
            for (uint32_t e = threadIdx.x; e < nver; e += kThreads) a.ver[e] = 0u;
            if (threadIdx.x == 0) a.ctrl->task_next = 0u;
        }
        if (a.mode & (kModeZ | kModeBsum)) {
            // every block of the group has read b's accumulator (before the
            // barrier that follows y): clear it for the next launch
            if (threadIdx.x == 0) a.ctrl->z_next = 0u;
            for (uint32_t j = threadIdx.x; j < a.x.ld; j += kThreads) stc(&a.bsum[j], 0.0);
        }
        __threadfence();
    }
}

}  // namespace hsp
