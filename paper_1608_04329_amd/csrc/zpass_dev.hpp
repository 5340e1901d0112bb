// The z pass: one read of X per sweep computes, for every row i,
//   eta_i = x_i beta                      (Section 5, z step i)
//   z_i ~ TN(eta_i, 1, y_i)               (Section 5, z step ii; Eq. 12)
//   b += x_i^T z_i                        (Section 5, beta step vi)
// Rows are full-conditionally independent (Eq. 8), so every row is drawn in
// parallel.  A wave owns a tile of R consecutive rows held in registers: each
// lane loads 16-byte vectors of every row (coalesced across the wave), the
// wave reduces the R dot products, lanes 0..R-1 draw one truncated normal
// each, and the same registers then feed x_i^T z_i.  X is read from HBM
// exactly once per sweep; eta and z never touch memory.
//
// Truncated normal, divergence-free: with y* = 2y - 1 and mu* = y* eta the
// draw is t ~ N(mu*, 1) restricted to t > 0 and z = y* t (the y* trick of
// Section 5 removes the sign divergence).  Every proposal evaluates both
// candidate samplers from the same two uniforms and selects one:
//   mu* > 0.47  Gaussian rejection: t = mu* + sqrt(-2 ln u1) cos(2 pi u2),
//               accept if t > 0;
//   otherwise   Robert (1995) exponential rejection with the optimal rate
//               theta = (-mu* + sqrt(mu*^2 + 4)) / 2 for the bound -mu* of
//               t - mu*: t = -ln(u1) / theta, accept if
//               u2 < exp(-(t - mu* - theta)^2 / 2) = exp(-(t - 1/theta)^2 / 2)
//               (theta (theta + mu*) = 1 makes the second form exact and free
//               of cancellation).
// So lanes on different branches run the same instructions.  Proposal a of
// row i uses Philox round a/2 (two proposals per call).
#pragma once
#include "hsp_internal.hpp"
#include "philox.hpp"
#include "sync_dev.hpp"

namespace hsp {

constexpr int kWPB = kThreads / kWave;  // waves per block
constexpr int kRedCols = kLdsDoubles / kWPB;  // columns per LDS reduction segment

template <int XT>
struct XTraits;
template <>
struct XTraits<0> {  // float32
    static constexpr int VEC = 4;
    static constexpr int BYTES = 4;
};
template <>
struct XTraits<1> {  // bfloat16
    static constexpr int VEC = 8;
    static constexpr int BYTES = 2;
};

#ifndef HSP_X_NONTEMPORAL
#define HSP_X_NONTEMPORAL 1
#endif
typedef unsigned int U32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t word_of(const uint4& v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// A tile's float32 sum of x_ij z_i, rounded to a multiple of 2^-24 (for
// |v| < 2^27).  Sums of such values below 2^29 in magnitude are exact in
// float64, so X^T z does not depend on which block summed which rows or in
// what order: the dynamically dealt tiles keep b bitwise reproducible.  The
// stored X has every column scaled into (-1, 1] by a power of two, so the
// grid is 2^-24 of the column's own scale, and the sums stay below 2^29 while
// sum_i |z_i| does.
__device__ __forceinline__ double on_grid(double v) {
    constexpr double kC = 0x1.8p28;  // 1.5 * 2^28: its float64 spacing is 2^-24
    return (v + kC) - kC;
}

template <int XT>
__device__ __forceinline__ float xelem(const uint4& v, int e) {
    if constexpr (XT == 0) {
        return __uint_as_float(word_of(v, e));
    } else {
        const uint32_t w = word_of(v, e >> 1);
        return (e & 1) ? __uint_as_float(w & 0xFFFF0000u) : __uint_as_float(w << 16);
    }
}

// One proposal from the uniforms (ua, ub): both candidates, one selected.
__device__ __forceinline__ void tn_candidate(float mu, bool gauss, float theta, float inv_theta,
                                             float ua, float ub, float& t, bool& acc) {
    const float L = -logf(ua);
    const float tg = fmaf(sqrtf(2.0f * L), cospif(2.0f * ub), mu);
    const float tr = L / theta;
    const float d = tr - inv_theta;
    const float rho = expf(-0.5f * d * d);
    t = gauss ? tg : tr;
    acc = gauss ? (tg > 0.0f) : (ub < rho);
}

// One tile of R rows of chain a (rows t R ..): eta = x_i beta (with wide
// rows, the block's four quarters added through LDS), the truncated-normal
// draws, and the tile's grid-rounded sums of x_ij z_i added into bacc.  bl
// holds beta (column-scaled, float32) on this lane's columns.
template <int XT, int KC, int R, bool WIDE>
__device__ __forceinline__ void z_tile(Args& a, uint32_t t, uint32_t ksweep,
                                       const float (&bl)[KC][XTraits<XT>::VEC],
                                       double (&bacc)[KC][XTraits<XT>::VEC], uint32_t& maxatt, bool& capped,
                                       uint32_t& parity, double* eta_lds) {
    constexpr int VEC = XTraits<XT>::VEC;
    constexpr int EB = XTraits<XT>::BYTES;
    constexpr int CW = kWave * VEC;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const uint32_t ld = a.x.ld;
    const uint32_t N = a.x.N;
    const char* __restrict__ Xb = static_cast<const char*>(a.x.X);
    const size_t row_bytes = (size_t)ld * EB;
    const uint32_t c0 = WIDE ? (uint32_t)wave * KC * CW : 0u;
    // The tile index is the same in every lane, so the row addresses are
    // scalar: each load is a scalar row base plus the lane's 32-bit column
    // offset.  Rows past the end are read as the last row and columns past
    // the row's end as its last chunk, so no load is predicated: those
    // elements meet a zero beta (no part in eta) and a zero z (rows past the
    // end are not drawn), and their column sums are never written out.
    const uint32_t row0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)t) * (uint32_t)R;
    uint32_t coff[KC];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) coff[kc] = min(c0 + kc * CW + lane * VEC, ld - VEC) * EB;
    uint4 xr[R][KC];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t ra = (uint64_t)(uintptr_t)Xb + (uint64_t)min(row0 + r, N - 1) * row_bytes;
        // (the builtin returns a signed int: each half goes through uint32_t
        // so that the low half is not sign-extended into the high one)
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(ra >> 32));
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)ra);
        const HSP_GLOBAL char* rp = reinterpret_cast<const HSP_GLOBAL char*>(((uint64_t)hi << 32) | (uint64_t)lo);
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const HSP_GLOBAL U32x4* src = reinterpret_cast<const HSP_GLOBAL U32x4*>(rp + coff[kc]);
#if HSP_X_NONTEMPORAL
            const U32x4 v = __builtin_nontemporal_load(src);
#else
            const U32x4 v = *src;
#endif
            xr[r][kc] = make_uint4(v.x, v.y, v.z, v.w);
        }
    }

    // eta for the R rows of the tile, reduced across the wave.  While a lane
    // holds more than one row, each exchange step halves them: the lane's bit
    // of the step picks the half it keeps, the partner lane keeps the other,
    // and each adds the half it receives, so the R rows cost R - 1 exchanges
    // instead of 6 R.  Once one row is left the steps are plain pairwise sums.
    // Lane l ends with the whole sum of row l >> (6 - log2 R).
    static_assert(R >= 1 && R <= kWave && (R & (R - 1)) == 0, "rows per tile: a power of two");
    constexpr int LR = R >= 32 ? 5 : R >= 16 ? 4 : R >= 8 ? 3 : R >= 4 ? 2 : R >= 2 ? 1 : 0;
    float s[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float acc = 0.0f;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc = fmaf(xelem<XT>(xr[r][kc], e), bl[kc][e], acc);
        s[r] = acc;
    }
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int off = kWave >> (st + 1);
        const int h = R >> (st + 1);  // rows kept after this step (0: one row left)
        if (h >= 1) {
            const bool up = (lane & off) != 0;
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const float send = up ? s[j] : s[j + h];
                const float keep = up ? s[j + h] : s[j];
                s[j] = keep + __shfl_xor(send, off);
            }
        } else {
            s[0] += __shfl_xor(s[0], off);
        }
    }
    float eta;
    if constexpr (WIDE) {
        // the four quarters' sums through LDS, added in wave order; the
        // two slots alternate, so one barrier per tile keeps a slot from
        // being rewritten before every wave has read it
        double* slotp = eta_lds + parity * (kWPB * R);
        if ((lane & ((1 << (6 - LR)) - 1)) == 0) slotp[wave * R + (lane >> (6 - LR))] = (double)s[0];
        __syncthreads();
        const int rr = lane < R ? lane : 0;
        float v = (float)slotp[rr];
#pragma unroll
        for (int w = 1; w < kWPB; ++w) v += (float)slotp[w * R + rr];
        eta = v;
        parity ^= 1u;
    } else {
        eta = __shfl(s[0], lane << (6 - LR));  // row `lane`'s sum, for lanes below R
    }

    // lane r < R draws z for row row0 + r: position first_row + row0 + r of
    // the stored X and y (X may arrive in row chunks), whose original row
    // index (the rows may have been reordered) sets its Philox counters
    // and its place in the debug outputs
    const uint32_t row = row0 + (uint32_t)lane;
    const bool active = lane < R && row < N;
    const uint32_t pos = a.first_row + row;
    const uint32_t grow = active ? (a.row_id ? a.row_id[pos] : pos) : 0u;
    const float ys = (active && a.y[pos]) ? 1.0f : -1.0f;
    const float mu = ys * eta;
    const bool gauss = mu > 0.47f;
    const float den = sqrtf(fmaf(mu, mu, 4.0f)) - mu;  // 2 theta
    const float theta = 0.5f * den;
    const float inv_theta = 2.0f / den;
    float zval = 0.0f;
    int32_t att = -1;
    bool done = !active;
    for (uint32_t round = 0; __ballot(!done) != 0ull; ++round) {
        if (!done) {
            const Words4 w = draw_words(a.seed, grow, ksweep, kTagZ, round, a.chain);
            float t0, t1;
            bool a0, a1;
            tn_candidate(mu, gauss, theta, inv_theta, u01f(w.w0), u01f(w.w1), t0, a0);
            tn_candidate(mu, gauss, theta, inv_theta, u01f(w.w2), u01f(w.w3), t1, a1);
            if (a0) {
                zval = ys * t0;
                att = (int32_t)(2 * round);
                done = true;
            } else if (a1) {
                zval = ys * t1;
                att = (int32_t)(2 * round + 1);
                done = true;
            } else if (round + 1 >= kMaxRounds) {
                zval = __builtin_nanf("");
                done = true;
                capped = true;
            }
        }
    }
    if (active && (!WIDE || wave == 0)) {
        maxatt = max(maxatt, (uint32_t)(att + 1));
        if (a.zdbg) {
            a.zdbg[grow] = zval;
            a.adbg[grow] = att | (gauss ? (1 << 30) : 0);
        }
    }

    // b += x_r^T z_r for the tile: R-term float sums, then float64
    float zr[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        zr[r] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zval), r));
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            float acc = 0.0f;
#pragma unroll
            for (int r = 0; r < R; ++r) acc = fmaf(zr[r], xelem<XT>(xr[r][kc], e), acc);
            bacc[kc][e] += on_grid((double)acc);
        }
}

// The z-pass role of the sweep kernel: block zrank of nz z-pass blocks.
// Short rows (WIDE false, see wide_chunks): each wave holds whole rows,
// KC chunks per lane, and takes tiles on its own.  Wider rows (WIDE): the
// block's four waves split every row into quarters of KC chunks per lane
// and take each tile together; their partial dot products meet in LDS and
// are added in wave order, so every wave holds the same eta and draws the
// same z, and each wave sums x_i^T z_i over its own quarter of the columns.
template <int XT, int KC, int R, bool WIDE = false>
__device__ __forceinline__ void zpass_role(Args& a, uint32_t zrank, uint32_t nz,
                                           uint32_t ksweep, double* red) {
    if (zrank >= nz) return;  // no z-pass work in this launch
    constexpr int VEC = XTraits<XT>::VEC;
    constexpr int CW = kWave * VEC;  // columns covered by one wave-wide 16-byte load

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const uint32_t ld = a.x.ld;
    const uint32_t N = a.x.N;
    const uint32_t c0 = WIDE ? (uint32_t)wave * KC * CW : 0u;  // first column of this wave's part

    float bl[KC][VEC];
    double bacc[KC][VEC];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const uint32_t col = c0 + kc * CW + lane * VEC + e;
            bl[kc][e] = col < ld ? a.beta32[col] : 0.0f;
            bacc[kc][e] = 0.0;
        }

    const uint32_t n_tiles = (N + R - 1) / R;
    // tiles are taken by waves, or for wide rows by whole blocks
    const uint32_t W = WIDE ? nz : nz * kWPB;
    uint32_t maxatt = 0;
    bool capped = false;
    uint32_t parity = 0;                // wide rows: LDS slot of the next tile's partial sums
    double* eta_lds = red + 8;          // [2][kWPB][R], after the unit slot

    auto tile = [&](uint32_t t) {
        z_tile<XT, KC, R, WIDE>(a, t, ksweep, bl, bacc, maxatt, capped, parity, eta_lds);
    };

    // A share of the tiles is dealt out statically, interleaved over all
    // waves; the rest go out in units of z_unit tiles to whichever block asks
    // next, so blocks on busier CUs do less of them.  Thread 0 reserves the
    // next unit before working on the current one.
    const uint32_t unit = a.z_unit;
    const uint32_t n_static = (uint32_t)((uint64_t)n_tiles * a.z_static_pct / 100 / W * W);
    for (uint32_t t = WIDE ? zrank : zrank * kWPB + wave; t < n_static; t += W) tile(t);
    if (n_static < n_tiles) {
        const uint32_t n_units = (n_tiles - n_static + unit - 1) / unit;
        double* slot = red;  // free until the reduction below
        if (threadIdx.x == 0) *slot = (double)atomicAdd(&a.ctrl->z_next, 1u);
        __syncthreads();
        uint32_t u = (uint32_t)*slot;
        __syncthreads();
        while (u < n_units) {
            uint32_t next = 0;
            if (threadIdx.x == 0) next = atomicAdd(&a.ctrl->z_next, 1u);
            for (uint32_t j = WIDE ? 0u : (uint32_t)wave; j < unit; j += WIDE ? 1u : (uint32_t)kWPB) {
                const uint32_t t = n_static + u * unit + j;
                if (t < n_tiles) tile(t);
            }
            if (threadIdx.x == 0) *slot = (double)next;
            __syncthreads();
            u = (uint32_t)*slot;
            __syncthreads();
        }
    }

    // wave statistics
    uint32_t m = maxatt;
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    const bool anycap = __ballot(capped) != 0ull;
    if (lane == 0) {
        if (m) atomicMax(&a.ctrl->max_attempts, m);
        if (anycap) atomicOr(&a.ctrl->err, kErrTnCap);
    }

    // block partial of X^T z: for wide rows, every wave's own columns; else
    // the waves' float64 sums added in wave order
    if constexpr (WIDE) {
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const uint32_t col = c0 + kc * CW + lane * VEC + e;
                if (col < ld) stc(&a.partial[(size_t)zrank * ld + col], bacc[kc][e]);
            }
    }
    for (uint32_t seg = 0; !WIDE && seg < ld; seg += kRedCols) {
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const uint32_t col = kc * CW + lane * VEC + e;
                if (col >= seg && col < seg + kRedCols && col < ld)
                    red[wave * kRedCols + (col - seg)] = bacc[kc][e];
            }
        __syncthreads();
        for (uint32_t c = threadIdx.x; c < kRedCols && seg + c < ld; c += kThreads) {
            double v = red[c];
#pragma unroll
            for (int w = 1; w < kWPB; ++w) v += red[w * kRedCols + c];
            stc(&a.partial[(size_t)zrank * ld + seg + c], v);
        }
        __syncthreads();
    }
    // This block's partial is complete.  The last of each group of kZGroup
    // consecutive blocks to finish adds the group's partials in block order
    // and adds the group sum into b's accumulator; the p-side waits for all
    // groups.  Partials and group sums move through coherent stores and
    // loads: every wave waits for its own stores before the block arrives.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const uint32_t grp = zrank / kZGroup;
    const uint32_t g0 = grp * kZGroup;
    const uint32_t gsize = min((uint32_t)kZGroup, nz - g0);
    if (threadIdx.x == 0) {
        const uint32_t old = atomicAdd(&a.zgrp_count[grp], 1u);
        const bool lst = old == gsize - 1;
        red[0] = lst ? 1.0 : 0.0;
    }
    __syncthreads();
    const bool last = red[0] != 0.0;
    __syncthreads();
    if (last) {
        for (uint32_t c = threadIdx.x; c < ld; c += kThreads) {
            double v[kZGroup];
#pragma unroll
            for (int r = 0; r < kZGroup; ++r)
                v[r] = (uint32_t)r < gsize ? ldc(&a.partial[(size_t)(g0 + r) * ld + c]) : 0.0;
            double s = v[0];
#pragma unroll
            for (int r = 1; r < kZGroup; ++r) s += v[r];
            // on the 2^-24 grid below 2^29 the float64 atomic additions are
            // exact, so the groups' order of arrival does not matter
            __hip_atomic_fetch_add(&a.bsum[c], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            // every block of the group has arrived
            __hip_atomic_store(&a.zgrp_count[grp], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicAdd(&a.ctrl->z_count, 1ull);
            // a launch without a p-side group (a chunk of rows) resets the
            // shared unit counter itself once every group has finished, i.e.
            // every block has left its claim loop
            if (a.gp == 0 && atomicAdd(&a.ctrl->z_done, 1u) == a.zgroups - 1) {
                __hip_atomic_store(&a.ctrl->z_done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&a.ctrl->z_next, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}


// A queue worker leaves chain a: the float64 sums of x_ij z_i over the units
// it finished there (each wave's, added in wave order) go into the chain's b
// accumulator, then its proposal statistics; once those additions are
// complete, the unit count goes into the chain's z_count.
template <int XT, int KC>
__device__ __forceinline__ void zq_flush(Args& a, double (&bacc)[KC][XTraits<XT>::VEC], uint32_t& maxatt,
                                         bool& capped, uint32_t units, double* red) {
    constexpr int VEC = XTraits<XT>::VEC;
    constexpr int CW = kWave * VEC;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const uint32_t ld = a.x.ld;
    for (uint32_t seg = 0; seg < ld; seg += kRedCols) {
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const uint32_t col = kc * CW + lane * VEC + e;
                if (col >= seg && col < seg + kRedCols && col < ld) red[wave * kRedCols + (col - seg)] = bacc[kc][e];
            }
        __syncthreads();
        for (uint32_t c = threadIdx.x; c < kRedCols && seg + c < ld; c += kThreads) {
            double v = red[c];
#pragma unroll
            for (int w = 1; w < kWPB; ++w) v += red[w * kRedCols + c];
            __hip_atomic_fetch_add(&a.bsum[seg + c], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int e = 0; e < VEC; ++e) bacc[kc][e] = 0.0;
    uint32_t m = maxatt;
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    const bool anycap = __ballot(capped) != 0ull;
    if (lane == 0) {
        if (m) atomicMax(&a.ctrl->max_attempts, m);
        if (anycap) atomicOr(&a.ctrl->err, kErrTnCap);
    }
    maxatt = 0;
    capped = false;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&a.ctrl->z_count, (unsigned long long)units);
}

// A worker block of a pack's shared z queue (rows of one wave each): the
// units of its home chain, then of whichever chain has most units left, until
// none are left anywhere.  Thread 0 reserves the next unit of the current
// chain before the block works on the present one.  Workers never wait on
// other blocks; the last one to finish clears the queue's counters for the
// next launch.
template <int XT, int KC, int R>
__device__ __forceinline__ void zqueue_role(const SweepArgs* const* tab, uint32_t home, double* red) {
    constexpr int VEC = XTraits<XT>::VEC;
    constexpr int CW = kWave * VEC;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    HSP_GLOBAL PackQ* q = ((Args*)tab[home])->zq;
    const uint32_t n = q->nchains;
    float bl[KC][VEC];
    double bacc[KC][VEC];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int e = 0; e < VEC; ++e) bacc[kc][e] = 0.0;
    uint32_t maxatt = 0, parity = 0;
    bool capped = false;

    uint32_t c = home;
    if (threadIdx.x == 0) red[0] = (double)atomicAdd(&q->next[c], 1u);
    __syncthreads();
    uint32_t u = (uint32_t)red[0];
    __syncthreads();
    for (;;) {
        const uint32_t nunits = q->units[c];
        if (u < nunits) {
            Args& a = *(Args*)tab[c];
            const uint32_t ksweep = a.ctrl->sweep + 1u;
            const uint32_t ld = a.x.ld, U = a.z_unit, n_tiles = (a.x.N + R - 1) / R;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const uint32_t col = kc * CW + lane * VEC + e;
                    bl[kc][e] = col < ld ? a.beta32[col] : 0.0f;
                }
            uint32_t finished = 0;
            while (u < nunits) {
                uint32_t nxt = 0;
                if (threadIdx.x == 0) nxt = atomicAdd(&q->next[c], 1u);
                for (uint32_t j = (uint32_t)wave; j < U; j += kWPB) {
                    const uint32_t t = u * U + j;
                    if (t < n_tiles) z_tile<XT, KC, R, false>(a, t, ksweep, bl, bacc, maxatt, capped, parity, nullptr);
                }
                ++finished;
                if (threadIdx.x == 0) red[0] = (double)nxt;
                __syncthreads();
                u = (uint32_t)red[0];
                __syncthreads();
            }
            zq_flush<XT, KC>(a, bacc, maxatt, capped, finished, red);
        }
        // the chain with most units left, the first of equals; a claim that
        // comes too late only sends the block back here
        if (wave == 0) {
            unsigned long long key = 0ull;
            for (uint32_t j = (uint32_t)lane; j < n; j += kWave) {
                const uint32_t nx = __hip_atomic_load(&q->next[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t un = q->units[j];
                const unsigned long long k =
                    un > nx ? ((unsigned long long)(un - nx) << 32) | (0xFFFFFFFFu - j) : 0ull;
                key = k > key ? k : key;
            }
#pragma unroll
            for (int off = kWave / 2; off >= 1; off >>= 1) {
                const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(key >> 32), off);
                const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)key, off);
                const unsigned long long o = ((unsigned long long)hi << 32) | lo;
                key = o > key ? o : key;
            }
            if (lane == 0) {
                if (key == 0ull) {
                    red[0] = -1.0;
                } else {
                    const uint32_t cc = 0xFFFFFFFFu - (uint32_t)key;
                    red[0] = (double)cc;
                    red[1] = (double)atomicAdd(&q->next[cc], 1u);
                }
            }
        }
        __syncthreads();
        const double r0 = red[0], r1 = red[1];
        __syncthreads();
        if (r0 < 0.0) break;
        c = (uint32_t)r0;
        u = (uint32_t)r1;
    }
    if (threadIdx.x == 0) red[0] = atomicAdd(&q->done, 1u) == q->workers - 1 ? 1.0 : 0.0;
    __syncthreads();
    if (red[0] != 0.0) {
        // every worker has made its last claim
        for (uint32_t j = threadIdx.x; j < n; j += kThreads)
            __hip_atomic_store(&q->next[j], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (threadIdx.x == 0) __hip_atomic_store(&q->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace hsp
