// The p-sized conditionals of Eq. (12), all in float64:
//   lambda_j^-2 ~ Exp(nu_j^-1 + tau^-2 beta_j^2 / 2)
//   tau^-2      ~ Gamma((p+1)/2, rate xi^-1 + sum_j lambda_j^-2 beta_j^2 / 2)
//   beta        ~ N(Q^-1 X^T z, Q^-1),  Q = X^T X + tau^-2 Lambda^-2
//   nu_j^-1     ~ Exp(1 + lambda_j^-2),   xi^-1 ~ Exp(1 + tau^-2)
// Exponential and gamma use the rate parameterisation fixed by Eq. (11);
// tau^-2 is the Gamma draw that the sampling step of Section 5 (Cheng 1977)
// produces, i.e. tau^2 is inverse-gamma.
#include <float.h>

#include "hsp_internal.hpp"
#include "philox.hpp"

namespace hsp {
namespace {

constexpr int kNB = 64;  // Cholesky / solve block

__device__ __forceinline__ uint32_t cur_sweep(const Ctrl* c) { return c->sweep + 1u; }

// ---- lambda^-2: one exponential per coordinate, by inversion ------------------
__global__ void lambda_kernel(PState s) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= s.p) return;
    const uint32_t k = cur_sweep(s.ctrl);
    const double bj = s.beta[j];
    double rate = s.nu_m1[j] + (*s.tau_m2) * bj * bj / 2.0;
    const bool clamp = !(rate >= DBL_MIN);
    if (clamp) rate = DBL_MIN;
    const Words4 w = draw_words(s.seed, j, k, kTagLambda, 0, s.chain);
    const double v = -log(u01d(w.w0)) / rate;
    s.lam_m2[j] = v;
    if (clamp) atomicAdd(&s.ctrl->clamps, 1ull);
    if (!isfinite(v)) atomicOr(&s.ctrl->err, kErrNonFinite);
}

// ---- tau^-2: one wave, Cheng's GB with one proposal per lane -------------------
// Proposal m = 64 * round + lane uses the uniforms of Philox round m/2 (words
// 0-1 for even m, 2-3 for odd m) of tag TAU; the lowest accepted m wins, which
// is exactly the first acceptance of the sequential algorithm.  (Section 5 uses
// 32 threads and a serial scan for the same purpose.)
__global__ __launch_bounds__(64) void tau_kernel(PState s) {
    const int lane = threadIdx.x;
    const uint32_t k = cur_sweep(s.ctrl);
    double acc = 0.0;
    for (uint32_t j = lane; j < s.p; j += kWave) acc += s.lam_m2[j] * s.beta[j] * s.beta[j];
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    const double rate = *s.xi_m1 + acc / 2.0;
    const double a = ((double)s.p + 1.0) / 2.0;
    const double A = 1.0 / sqrt(2.0 * a - 1.0);
    const double B = a - log(4.0);
    const double C = a + 1.0 / A;
    const double D = 1.0 + log(4.5);
    double g = __builtin_nan("");
    for (uint32_t round = 0; round < (1u << 16); ++round) {
        const uint32_t m = round * kWave + lane;
        const Words4 w = draw_words(s.seed, 0, k, kTagTau, m >> 1, s.chain);
        const double u1 = u01d((m & 1u) ? w.w2 : w.w0);
        const double u2 = u01d((m & 1u) ? w.w3 : w.w1);
        const double V = A * log(u1 / (1.0 - u1));
        const double X = a * exp(V);
        const double Z = u1 * u1 * u2;
        const double R = B + C * V - X;
        const bool ok = (R + D - 4.5 * Z >= 0.0) || (R >= log(Z));
        const unsigned long long mask = __ballot(ok);
        if (mask) {
            g = __shfl(X, (int)(__ffsll((long long)mask) - 1));
            break;
        }
    }
    if (lane == 0) {
        const double t = g / rate;
        *s.tau_m2 = t;
        if (!isfinite(t) || !(t > 0.0)) atomicOr(&s.ctrl->err, kErrNonFinite);
    }
}

// ---- nu^-1 and xi^-1 ----------------------------------------------------------
__global__ void nuxi_kernel(PState s) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t k = cur_sweep(s.ctrl);
    if (j < s.p) {
        const Words4 w = draw_words(s.seed, j, k, kTagNu, 0, s.chain);
        s.nu_m1[j] = -log(u01d(w.w0)) / (1.0 + s.lam_m2[j]);
    }
    if (j == 0) {
        const Words4 w = draw_words(s.seed, 0, k, kTagXi, 0, s.chain);
        *s.xi_m1 = -log(u01d(w.w0)) / (1.0 + *s.tau_m2);
    }
}

// ---- register-resident triangular solves for one wave ---------------------
// The right-hand side lives in registers, lane l holding entries l, l+64, ...;
// U is read from LDS (row-major, leading dimension ldu).  Forward: U^T x = r;
// backward: U x = r.  x overwrites r.
template <int PL>
__device__ __forceinline__ double lane_get(const double (&r)[PL], uint32_t i) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < PL; ++q) v = (i / kWave == (uint32_t)q) ? __shfl(r[q], (int)(i % kWave)) : v;
    return v;
}

template <int PL>
__device__ void wave_solve_forward(const double* U, uint32_t ldu, uint32_t p, double (&r)[PL]) {
    const int lane = threadIdx.x & (kWave - 1);
    for (uint32_t i = 0; i < p; ++i) {
        const double xi = lane_get<PL>(r, i) / U[i * ldu + i];
#pragma unroll
        for (int q = 0; q < PL; ++q) {
            const uint32_t j = q * kWave + lane;
            if (j == i) r[q] = xi;
            else if (j > i && j < p) r[q] -= U[i * ldu + j] * xi;
        }
    }
}

template <int PL>
__device__ void wave_solve_backward(const double* U, uint32_t ldu, uint32_t p, double (&r)[PL]) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int ii = (int)p - 1; ii >= 0; --ii) {
        const uint32_t i = (uint32_t)ii;
        const double xi = lane_get<PL>(r, i) / U[i * ldu + i];
#pragma unroll
        for (int q = 0; q < PL; ++q) {
            const uint32_t j = q * kWave + lane;
            if (j == i) r[q] = xi;
            else if (j < i) r[q] -= U[j * ldu + i] * xi;
        }
    }
}

// ---- beta for p <= 128: the whole step in one block, Q in LDS -----------------
// Right-looking Cholesky with the row scaling deferred: step c subtracts
// A[c][i] A[c][j] / A[c][c] from the trailing upper triangle (row c itself is
// never written after its step), and row c is scaled by 1/sqrt(A[c][c]) at the
// end, giving Q = U^T U with U upper.  Then, in one wave: s ~ N(0, I),
// U v = s (Cov v = Q^-1), U^T w = b, U mu = w, beta = mu + v.
constexpr uint32_t kSmallP = 128;

__global__ __launch_bounds__(1024) void beta_small_kernel(PState s) {
    extern __shared__ double U[];  // p x (p + 1)
    const uint32_t p = s.p, ldu = p + 1;
    const uint32_t k = cur_sweep(s.ctrl);
    const double tau = *s.tau_m2;
    for (uint32_t idx = threadIdx.x; idx < p * p; idx += blockDim.x) {
        const uint32_t i = idx / p, j = idx % p;
        U[i * ldu + j] = s.G[idx] + (i == j ? tau * s.lam_m2[i] : 0.0);
    }
    __syncthreads();
    bool bad = false;
    for (uint32_t c = 0; c < p; ++c) {
        const double d = U[c * ldu + c];
        if (!(d > 0.0)) bad = true;
        const double inv = 1.0 / d;
        const uint32_t m = p - c - 1;
        for (uint32_t idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
            const uint32_t i = c + 1 + idx / m, j = c + 1 + idx % m;
            if (j >= i) U[i * ldu + j] -= U[c * ldu + i] * inv * U[c * ldu + j];
        }
        __syncthreads();
        if (bad) break;
    }
    if (bad) {
        if (threadIdx.x == 0) {
            atomicOr(&s.ctrl->err, kErrNotPD);
            for (uint32_t c = 0; c < p; ++c)
                if (!(U[c * ldu + c] > 0.0)) { atomicCAS(&s.ctrl->chol_info, 0, (int)(c + 1)); break; }
        }
        return;
    }
    // scale rows: U[c][j] = A[c][j] / sqrt(A[c][c]) (the strict lower part is never read)
    for (uint32_t idx = threadIdx.x; idx < p * p; idx += blockDim.x) {
        const uint32_t i = idx / p, j = idx % p;
        if (j > i) U[i * ldu + j] = U[i * ldu + j] / sqrt(U[i * ldu + i]);
    }
    __syncthreads();
    if (threadIdx.x < p) U[threadIdx.x * ldu + threadIdx.x] = sqrt(U[threadIdx.x * ldu + threadIdx.x]);
    __syncthreads();
    if (threadIdx.x >= kWave) return;

    const int lane = threadIdx.x;
    constexpr int PL = kSmallP / kWave;
    double v[PL], w[PL];
#pragma unroll
    for (int q = 0; q < PL; ++q) {
        const uint32_t j = q * kWave + lane;
        v[q] = 0.0;
        w[q] = 0.0;
        if (j < p) {
            const Words4 wd = draw_words(s.seed, j, k, kTagBetaS, 0, s.chain);
            v[q] = box_muller_d(u01d(wd.w0), u01d(wd.w1));
            w[q] = s.b[j];
        }
    }
    wave_solve_backward<PL>(U, ldu, p, v);
    wave_solve_forward<PL>(U, ldu, p, w);
    wave_solve_backward<PL>(U, ldu, p, w);
    bool nonfinite = false;
#pragma unroll
    for (int q = 0; q < PL; ++q) {
        const uint32_t j = q * kWave + lane;
        if (j < p) {
            const double bj = w[q] + v[q];
            s.beta[j] = bj;
            s.beta32[j] = (float)bj;
            if (!isfinite(bj)) nonfinite = true;
        }
    }
    if (__ballot(nonfinite) && lane == 0) atomicOr(&s.ctrl->err, kErrNonFinite);
}

// ---- beta for p > 128: blocked Cholesky in global memory ---------------------
// Q (upper triangle) is built in A, then for every block column kb:
//   panel : factor the 64 x 64 diagonal block in LDS and solve
//           U_kk^T U_kj = A_kj for the blocks j > k of block row k;
//   update: A_ij -= U_ki^T U_kj for all trailing blocks k < i <= j.
__global__ void qbuild_kernel(PState s) {
    const uint32_t p = s.p;
    const double tau = *s.tau_m2;
    const size_t n = (size_t)p * p;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)(idx / p), j = (uint32_t)(idx % p);
        if (j >= i) s.A[idx] = s.G[idx] + (i == j ? tau * s.lam_m2[i] : 0.0);
    }
}

__global__ __launch_bounds__(256) void chol_panel_kernel(double* A, double* Ud, uint32_t p,
                                                         uint32_t kb, Ctrl* ctrl) {
    __shared__ double D[kNB][kNB + 1];
    __shared__ double rs[kNB];
    const uint32_t k0 = kb * kNB;
    const uint32_t bs = min((uint32_t)kNB, p - k0);
    const uint32_t jb = kb + blockIdx.x;
    const uint32_t j0 = jb * kNB;
    const uint32_t ws = min((uint32_t)kNB, p - j0);
    const int tid = threadIdx.x;

    // diagonal block, padded with the identity beyond the matrix edge
    for (int idx = tid; idx < kNB * kNB; idx += 256) {
        const int i = idx / kNB, j = idx % kNB;
        double v;
        if ((uint32_t)i < bs && (uint32_t)j < bs) v = (j >= i) ? A[(size_t)(k0 + i) * p + k0 + j] : 0.0;
        else v = (i == j) ? 1.0 : 0.0;
        D[i][j] = v;
    }
    __syncthreads();
    bool bad = false;
    for (int c = 0; c < kNB; ++c) {
        const double d = D[c][c];
        if (!(d > 0.0)) bad = true;
        const double inv = 1.0 / d;
        const int m = kNB - c - 1;
        for (int idx = tid; idx < m * m; idx += 256) {
            const int i = c + 1 + idx / m, j = c + 1 + idx % m;
            if (j >= i) D[i][j] -= D[c][i] * inv * D[c][j];
        }
        __syncthreads();
        if (bad) break;
    }
    if (bad) {
        if (tid == 0 && blockIdx.x == 0) {
            atomicOr(&ctrl->err, kErrNotPD);
            for (int c = 0; c < kNB; ++c)
                if (!(D[c][c] > 0.0)) { atomicCAS(&ctrl->chol_info, 0, (int)(k0 + c + 1)); break; }
        }
        return;
    }
    if (tid < kNB) rs[tid] = sqrt(D[tid][tid]);
    __syncthreads();
    for (int idx = tid; idx < kNB * kNB; idx += 256) {
        const int i = idx / kNB, j = idx % kNB;
        if (j > i) D[i][j] = D[i][j] / rs[i];
    }
    __syncthreads();
    if (tid < kNB) D[tid][tid] = rs[tid];
    __syncthreads();

    if (blockIdx.x == 0) {
        // the other blocks of this launch still read A_kk, so the factor of the
        // diagonal block goes to its own buffer (identity-padded, lower part 0)
        for (int idx = tid; idx < kNB * kNB; idx += 256) {
            const int i = idx / kNB, j = idx % kNB;
            Ud[(size_t)kb * kNB * kNB + idx] = (j >= i) ? D[i][j] : 0.0;
        }
        return;
    }
    // U_kk^T X = A_kj, one column of X per lane of wave 0, kept in registers
    if (tid >= kNB) return;
    const int c = tid;
    double x[kNB];
#pragma unroll
    for (int i = 0; i < kNB; ++i)
        x[i] = ((uint32_t)i < bs && (uint32_t)c < ws) ? A[(size_t)(k0 + i) * p + j0 + c] : 0.0;
#pragma unroll
    for (int i = 0; i < kNB; ++i) {
        const double xi = x[i] / D[i][i];
        x[i] = xi;
#pragma unroll
        for (int m = i + 1; m < kNB; ++m) x[m] -= D[i][m] * xi;
    }
    if ((uint32_t)c < ws)
#pragma unroll
        for (int i = 0; i < kNB; ++i)
            if ((uint32_t)i < bs) A[(size_t)(k0 + i) * p + j0 + c] = x[i];
}

__global__ __launch_bounds__(256) void chol_update_kernel(double* A, uint32_t p, uint32_t kb,
                                                          uint32_t nt) {
    constexpr int KS = 32;
    __shared__ double Ui[KS][kNB + 1];
    __shared__ double Uj[KS][kNB + 1];
    // block -> trailing tile (ib, jb), kb < ib <= jb < nt
    const uint32_t m = nt - kb - 1;
    uint32_t idx = blockIdx.x, r = 0;
    while (idx >= m - r) { idx -= m - r; ++r; }
    const uint32_t ib = kb + 1 + r, jb = ib + idx;
    const uint32_t k0 = kb * kNB, i0 = ib * kNB, j0 = jb * kNB;
    const uint32_t bs = min((uint32_t)kNB, p - k0);
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    double acc[4][4] = {};
    for (uint32_t mm = 0; mm < bs; mm += KS) {
        for (int e = tid; e < KS * kNB; e += 256) {
            const int q = e / kNB, c = e % kNB;
            const uint32_t row = k0 + mm + q;
            const bool rok = (mm + q) < bs;
            Ui[q][c] = (rok && i0 + c < p) ? A[(size_t)row * p + i0 + c] : 0.0;
            Uj[q][c] = (rok && j0 + c < p) ? A[(size_t)row * p + j0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < KS; ++q) {
            double ai[4], aj[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                ai[t] = Ui[q][ty * 4 + t];
                aj[t] = Uj[q][tx * 4 + t];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[t][u] += ai[t] * aj[u];
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t i = i0 + ty * 4 + t, j = j0 + tx * 4 + u;
            if (i < p && j < p && j >= i) A[(size_t)i * p + j] -= acc[t][u];
        }
}

// Triangular solve with the upper factor in A (row-major, ld p) by one block:
// trans = 1: U^T x = r (forward), trans = 0: U x = r (backward).  The
// right-hand side stays in LDS; each 64-row diagonal block is solved by wave 0
// from LDS, then every wave applies that block's contribution to the rest.
__global__ __launch_bounds__(1024) void trsv_kernel(const double* __restrict__ U,
                                                    const double* __restrict__ Ud, uint32_t p,
                                                    const double* __restrict__ r,
                                                    double* __restrict__ x, int trans) {
    __shared__ double rhs[kMaxP];
    __shared__ double Dg[kNB][kNB + 1];
    __shared__ double xs[kNB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
    for (uint32_t j = tid; j < p; j += blockDim.x) rhs[j] = r[j];
    __syncthreads();
    const uint32_t nb = (p + kNB - 1) / kNB;
    for (uint32_t step = 0; step < nb; ++step) {
        const uint32_t ib = trans ? step : nb - 1 - step;
        const uint32_t i0 = ib * kNB, bs = min((uint32_t)kNB, p - i0);
        for (uint32_t e = tid; e < kNB * kNB; e += blockDim.x) Dg[e / kNB][e % kNB] = Ud[(size_t)ib * kNB * kNB + e];
        __syncthreads();
        if (wave == 0) {
            double rl = (uint32_t)lane < bs ? rhs[i0 + lane] : 0.0;
            double xl = 0.0;
            if (trans) {
                for (int i = 0; i < kNB; ++i) {
                    const double xi = __shfl(rl, i) / Dg[i][i];
                    if (lane == i) xl = xi;
                    else if (lane > i) rl -= Dg[i][lane] * xi;
                }
            } else {
                for (int i = kNB - 1; i >= 0; --i) {
                    const double xi = __shfl(rl, i) / Dg[i][i];
                    if (lane == i) xl = xi;
                    else if (lane < i) rl -= Dg[lane][i] * xi;
                }
            }
            xs[lane] = (uint32_t)lane < bs ? xl : 0.0;
            if ((uint32_t)lane < bs) x[i0 + lane] = xl;
        }
        __syncthreads();
        if (trans) {
            // rhs[j] -= sum_i U[i0+i][j] x_i for j beyond the block
            for (uint32_t j = i0 + bs + tid; j < p; j += blockDim.x) {
                double acc = 0.0;
                for (uint32_t i = 0; i < bs; ++i) acc += U[(size_t)(i0 + i) * p + j] * xs[i];
                rhs[j] -= acc;
            }
        } else {
            // rhs[j] -= sum_i U[j][i0+i] x_i for j before the block: one wave per row
            for (uint32_t j = wave; j < i0; j += nwaves) {
                double v = (uint32_t)lane < bs ? U[(size_t)j * p + i0 + lane] * xs[lane] : 0.0;
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
                if (lane == 0) rhs[j] -= v;
            }
        }
        __syncthreads();
    }
}

__global__ void noise_kernel(PState s, double* out) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= s.p) return;
    const Words4 w = draw_words(s.seed, j, cur_sweep(s.ctrl), kTagBetaS, 0, s.chain);
    out[j] = box_muller_d(u01d(w.w0), u01d(w.w1));
}

__global__ void beta_combine_kernel(PState s, const double* mu, const double* v) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= s.p) return;
    const double bj = mu[j] + v[j];
    s.beta[j] = bj;
    s.beta32[j] = (float)bj;
    if (!isfinite(bj)) atomicOr(&s.ctrl->err, kErrNonFinite);
}

// ---- recording, sweep counter, test hook ----------------------------------------
__global__ void record_kernel(PState s, double* ring_beta, double* ring_tau, double* ring_lam,
                              uint32_t thin, uint32_t capacity) {
    const uint32_t k = cur_sweep(s.ctrl);
    const uint32_t since = k - s.ctrl->draw_base;
    if (since % thin != 0) return;
    const uint32_t d = since / thin - 1u;
    const size_t slot = d % capacity;
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < s.p) {
        ring_beta[slot * s.p + j] = s.beta[j];
        if (ring_lam) ring_lam[slot * s.p + j] = s.lam_m2[j];
    }
    if (j == 0) ring_tau[slot] = *s.tau_m2;
}

__global__ void advance_kernel(Ctrl* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) c->sweep = c->sweep + 1u;
}

__global__ void philox_test_kernel(uint64_t seed, const uint32_t* ctr, uint32_t n, uint32_t* out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Words4 w = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3],
                                   (uint32_t)seed, (uint32_t)(seed >> 32));
    out[4 * i] = w.w0;
    out[4 * i + 1] = w.w1;
    out[4 * i + 2] = w.w2;
    out[4 * i + 3] = w.w3;
}

inline unsigned blocks_for(uint32_t n, unsigned t) { return (n + t - 1) / t; }

}  // namespace

hipError_t lambda_launch(const PState& s, hipStream_t st) {
    hipLaunchKernelGGL(lambda_kernel, dim3(blocks_for(s.p, 256)), dim3(256), 0, st, s);
    return hipGetLastError();
}

hipError_t tau_launch(const PState& s, hipStream_t st) {
    hipLaunchKernelGGL(tau_kernel, dim3(1), dim3(64), 0, st, s);
    return hipGetLastError();
}

hipError_t nuxi_launch(const PState& s, hipStream_t st) {
    hipLaunchKernelGGL(nuxi_kernel, dim3(blocks_for(s.p, 256)), dim3(256), 0, st, s);
    return hipGetLastError();
}

bool beta_small_fits(uint32_t p, size_t max_lds) {
    return p <= kSmallP && sizeof(double) * p * (p + 1) <= max_lds;
}

hipError_t pside_prepare(size_t max_lds) {
    const size_t want = sizeof(double) * kSmallP * (kSmallP + 1);
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&beta_small_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(want < max_lds ? want : max_lds));
}

hipError_t beta_launch(const PState& s, hipStream_t st) {
    const uint32_t p = s.p;
    if (s.small_lds_ok) {
        const size_t lds = sizeof(double) * p * (p + 1);
        hipLaunchKernelGGL(beta_small_kernel, dim3(1), dim3(1024), lds, st, s);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(qbuild_kernel, dim3(256), dim3(256), 0, st, s);
    const uint32_t nt = (p + kNB - 1) / kNB;
    for (uint32_t kb = 0; kb < nt; ++kb) {
        hipLaunchKernelGGL(chol_panel_kernel, dim3(nt - kb), dim3(256), 0, st, s.A, s.Ud, p, kb,
                           s.ctrl);
        const uint32_t m = nt - kb - 1;
        if (m)
            hipLaunchKernelGGL(chol_update_kernel, dim3(m * (m + 1) / 2), dim3(256), 0, st, s.A, p,
                               kb, nt);
    }
    double* sv = s.vec;          // s, then v
    double* w = s.vec + p;       // U^T w = b
    double* mu = s.vec + 2 * p;  // U mu = w
    double* v = s.vec + 3 * p;
    hipLaunchKernelGGL(noise_kernel, dim3(blocks_for(p, 256)), dim3(256), 0, st, s, sv);
    hipLaunchKernelGGL(trsv_kernel, dim3(1), dim3(1024), 0, st, (const double*)s.A,
                       (const double*)s.Ud, p, (const double*)sv, v, 0);
    hipLaunchKernelGGL(trsv_kernel, dim3(1), dim3(1024), 0, st, (const double*)s.A,
                       (const double*)s.Ud, p, (const double*)s.b, w, 1);
    hipLaunchKernelGGL(trsv_kernel, dim3(1), dim3(1024), 0, st, (const double*)s.A,
                       (const double*)s.Ud, p, (const double*)w, mu, 0);
    hipLaunchKernelGGL(beta_combine_kernel, dim3(blocks_for(p, 256)), dim3(256), 0, st, s,
                       (const double*)mu, (const double*)v);
    return hipGetLastError();
}

hipError_t record_launch(const PState& s, double* ring_beta, double* ring_tau, double* ring_lam,
                         uint32_t thin, uint32_t capacity, hipStream_t st) {
    hipLaunchKernelGGL(record_kernel, dim3(blocks_for(s.p, 256)), dim3(256), 0, st, s, ring_beta,
                       ring_tau, ring_lam, thin, capacity);
    return hipGetLastError();
}

hipError_t advance_launch(Ctrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, st, ctrl);
    return hipGetLastError();
}

hipError_t philox_test_launch(uint64_t seed, const uint32_t* ctr, uint32_t n, uint32_t* out,
                              hipStream_t st) {
    hipLaunchKernelGGL(philox_test_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, seed, ctr,
                       n, out);
    return hipGetLastError();
}

}  // namespace hsp
