// The multi-chain z pass: up to kMcChains chains on one bfloat16 design
// share a single read of X per sweep.  For every row i and chain c it
// computes (Section 5, z steps i-ii and beta step vi, for many chains)
//   eta_ic = x_i beta_c,  z_ic ~ TN(eta_ic, 1, y_i),  b_c += x_i^T z_ic,
// i.e. the two matrix-vector products of the single-chain pass become
// products with a 16-column right-hand side: H = X B and b = X^T Z, on the
// bfloat16 matrix cores.
//
// Operands.  X is bfloat16 already (exact).  beta and z are float32: each is
// split into bfloat16 hi + lo (round to nearest twice), so each product is two
// matrix-core operations, the residual |v - hi - lo| <= 2^-18 |v|; the
// products are exact in float32 and accumulate in float32.
//
// Layout (one block = 4 waves, tiles of kMcRows = 16 rows): wave w owns the
// 32-column steps [w KS, (w + 1) KS) of every row.
//  * X beta: v_mfma_f32_16x16x32_bf16 with A = the X tile (lane l: row l % 16,
//    columns 8 (l / 16) .. + 7 of the step, one 16-byte load) and B = beta
//    (lane l: chain l % 16, the same 8 columns).  The four waves' partial
//    sums meet in LDS, summed in wave order.
//  * The TN draw: thread t draws row t / 16 for chain t % 16 (the same
//    divergence-free sampler and Philox counters as the single-chain pass).
//  * X^T z needs the tile with rows, not columns, along each lane.  The same
//    registers are transposed on the matrix cores by a product with an
//    identity block (x 1 plus zeros: exact): lane l then holds rows
//    4 (l / 16) .. + 3 of one column, which is the A operand of
//    v_mfma_f32_16x16x16bf16_1k against B = z (lane l: chain l % 16, the
//    same four rows).  D (16 columns x 16 chains) accumulates over a unit of
//    kMcUnit tiles in float32.
//  * At the end of a unit, each D entry is rounded to the 2^-24 grid (in the
//    stored, column-scaled units) and added into the block's float64 partial;
//    sums of grid values are exact in any order, so units may be claimed
//    dynamically and the group sums added into each chain's X^T z
//    accumulator with float64 atomics while every run stays bit-reproducible.
//
// The pass is a launch of its own; the chains' p-side groups run in the next
// launch and take b from the accumulators (the kernel boundary orders them).
#pragma once
#include "hsp_internal.hpp"
#include "philox.hpp"
#include "sync_dev.hpp"
#include "zpass_dev.hpp"

namespace hsp {

typedef __bf16 Bf16x8 __attribute__((ext_vector_type(8)));
typedef short Bf16x4 __attribute__((ext_vector_type(4)));  // four bfloat16 bit patterns
typedef float F32x4 __attribute__((ext_vector_type(4)));

using McView = const HSP_CONST McArgs;

__device__ __forceinline__ uint32_t bf16_rne_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

// v = hi + lo + r with |r| <= 2^-18 |v| (finite v).
__device__ __forceinline__ void split_bf16(float v, uint32_t& hi, uint32_t& lo) {
    hi = bf16_rne_bits(v);
    lo = bf16_rne_bits(v - bf16_value(hi));
}

__device__ __forceinline__ Bf16x8 as_bf16x8(const U32x4& v) { return __builtin_bit_cast(Bf16x8, v); }

// Four float32 values that are bfloat16 numbers, as their bit patterns.
__device__ __forceinline__ Bf16x4 pack_exact_bf16(const F32x4& t) {
    Bf16x4 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = (short)(__float_as_uint(t[i]) >> 16);
    return r;
}

// LDS of the pass (floats): red [4 waves][16 rows][16 chains], z [16 rows][16
// chains], the claimed unit, then beta's high and low parts as bfloat16,
// each [column / 8][chain][8] (one 16-byte read per lane, consecutive lanes
// on consecutive addresses).
constexpr int kMcRedFloats = 4 * kMcRows * kMcChains;
constexpr int kMcZFloats = kMcRows * kMcChains;
constexpr int kMcBetaOffFloats = kMcRedFloats + kMcZFloats + 64;
constexpr int kMcBetaChunks = kMcMaxLd / 8 * kMcChains;  // 16-byte chunks of one part
constexpr int kMcLdsDoubles = (kMcBetaOffFloats + 2 * kMcBetaChunks * 4) / 2;

template <int KS>
__device__ void mc_role(McView& m, uint32_t rank, double* lds) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int q = lane >> 4, n = lane & 15;
    const uint32_t ld = m.x.ld, N = m.x.N, C = m.nchains;
    float* red = reinterpret_cast<float*>(lds);
    float* zl = red + kMcRedFloats;
    uint32_t* slot = reinterpret_cast<uint32_t*>(zl + kMcZFloats);
    U32x4* bhi_lds = reinterpret_cast<U32x4*>(red + kMcBetaOffFloats);
    U32x4* blo_lds = bhi_lds + kMcBetaChunks;
    const char* __restrict__ Xb = static_cast<const char*>(m.x.X);
    const size_t row_bytes = (size_t)ld * 2;
    const uint32_t ks0 = (uint32_t)wave * KS;  // this wave's first 32-column step

    // Chain n of this lane (the columns of the products; thread t's TN draws
    // are for chain t % 16 = n as well).
    const bool live = (uint32_t)n < C;
    uint64_t seed = 0;
    uint32_t cid = 0, kk = 0;
    HSP_GLOBAL const float* b32 = nullptr;
    HSP_GLOBAL float* zdbg = nullptr;
    HSP_GLOBAL int32_t* adbg = nullptr;
    HSP_GLOBAL Ctrl* ctrl = nullptr;
    if (live) {
        Args& a = *(Args*)m.chain[n];
        seed = a.seed;
        cid = a.chain;
        ctrl = a.ctrl;
        kk = ctrl->sweep + 1u;
        b32 = a.beta32;
        zdbg = a.zdbg;
        adbg = a.adbg;
    }

    // beta of chain n on this lane's columns, split, into LDS (every block
    // holds all of it)
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        U32x4 hv, lv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint32_t h[2], l[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const uint32_t col = 32u * (ks0 + s) + 8u * q + 2u * i + e;
                const float v = (live && col < ld) ? b32[col] : 0.0f;
                split_bf16(v, h[e], l[e]);
            }
            hv[i] = h[0] | h[1] << 16;
            lv[i] = l[0] | l[1] << 16;
        }
        bhi_lds[(4u * (ks0 + s) + q) * kMcChains + n] = hv;
        blo_lds[(4u * (ks0 + s) + q) * kMcChains + n] = lv;
    }
    // identity blocks for the transposition: I_h[k][c] = (k == 16 h + c)
    Bf16x8 idm[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        U32x4 v;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k0 = 8 * q + 2 * i;
            const uint32_t lo16 = k0 == 16 * h + n ? 0x3F80u : 0u;
            const uint32_t hi16 = k0 + 1 == 16 * h + n ? 0x3F80u : 0u;
            v[i] = lo16 | hi16 << 16;
        }
        idm[h] = as_bf16x8(v);
    }

    const uint32_t n_tiles = (N + kMcRows - 1) / kMcRows;
    const uint32_t n_units = (n_tiles + kMcUnit - 1) / kMcUnit;
    HSP_GLOBAL uint32_t* unit_next = m.count + m.zgroups + 32;
    uint32_t maxatt = 0;
    bool capped = false, wrote = false;

    // tile t's X (16-byte loads) and the outcome of the row this thread draws
    U32x4 xr[KS];
    uint32_t ypre = 0;
    // Every lane loads, with no branch: a row past the last reads the last
    // row (its z is 0, so it adds nothing to X^T z) and a column past the
    // last reads the row's last 16 bytes (beta is 0 there, and those columns
    // of the partial are never read), so each product is the one zeros give.
    auto load_tile = [&](uint32_t t) {
        ypre = (uint32_t)m.y[min(t * kMcRows + (threadIdx.x >> 4), N - 1u)];
        const char* rowp = Xb + (size_t)min(t * kMcRows + (uint32_t)n, N - 1u) * row_bytes;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const uint32_t col = min(32u * (ks0 + s) + 8u * q, ld - 8u);
            xr[s] = __builtin_nontemporal_load(reinterpret_cast<const U32x4*>(rowp + (size_t)col * 2));
        }
    };

    F32x4 db[KS][2];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) db[s][h] = F32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // a unit's X^T z into the block's float64 partial: D entry r of step
    // (s, h) is column 32 (ks0 + s) + 16 h + 4 q + r of chain n.  Every lane
    // stores all of its entries (rows of the partial span every column the
    // waves cover, and D is zero past ld and for chains past C), with no
    // branch between the stores, so they are all in flight together; the
    // earlier sums are loaded four steps at a time, likewise.
    auto flush = [&]() {
        HSP_GLOBAL double* dst = m.partial + ((size_t)rank * kMcChains + n) * m.pstride;
#pragma unroll
        for (int s0 = 0; s0 < KS; s0 += 4) {
            double old[4][2][4];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        old[s][h][r] = wrote ? ldc(dst + 32u * (ks0 + s0 + s) + 16u * h + 4u * q + r) : 0.0;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double v = on_grid((double)db[s0 + s][h][r]);
                        stc(dst + 32u * (ks0 + s0 + s) + 16u * h + 4u * q + r, wrote ? old[s][h][r] + v : v);
                    }
        }
        wrote = true;
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int h = 0; h < 2; ++h) db[s][h] = F32x4{0.0f, 0.0f, 0.0f, 0.0f};
    };

    // the TN draw of (row t / 16, chain t % 16) reads its eta from red
    const uint32_t mrow = threadIdx.x >> 4;
    if (threadIdx.x == 0) *slot = atomicAdd(unit_next, 1u);
    __syncthreads();  // also orders the beta low parts in LDS before any use
    uint32_t u = *slot;
    __syncthreads();
    while (u < n_units) {
        uint32_t next = 0;
        if (threadIdx.x == 0) next = atomicAdd(unit_next, 1u);
        const uint32_t t0 = u * kMcUnit, t1 = min(n_tiles, t0 + kMcUnit);
        load_tile(t0);
        for (uint32_t t = t0; t < t1; ++t) {
            // X beta for the 16 chains, and the transposed tile
            F32x4 de = {0.0f, 0.0f, 0.0f, 0.0f};
            const uint32_t ycur = ypre;
            Bf16x4 tt[KS][2];
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const Bf16x8 A = as_bf16x8(xr[s]);
                const Bf16x8 bhi = as_bf16x8(bhi_lds[(4u * (ks0 + s) + q) * kMcChains + n]);
                const Bf16x8 blo = as_bf16x8(blo_lds[(4u * (ks0 + s) + q) * kMcChains + n]);
                de = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, bhi, de, 0, 0, 0);
                de = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, blo, de, 0, 0, 0);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const F32x4 tr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        A, idm[h], F32x4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
                    tt[s][h] = pack_exact_bf16(tr);
                }
            }
            if (t + 1 < t1) load_tile(t + 1);  // in flight during the draws
#pragma unroll
            for (int r = 0; r < 4; ++r) red[(wave * kMcRows + 4 * q + r) * kMcChains + n] = de[r];
            __syncthreads();

            // z for (row, chain n)
            const uint32_t row = t * kMcRows + mrow;
            const bool active = live && row < N;
            float eta = 0.0f;
#pragma unroll
            for (int w = 0; w < kWPB; ++w) eta += red[(w * kMcRows + mrow) * kMcChains + n];
            const float ys = (active && ycur) ? 1.0f : -1.0f;
            const float mu = ys * eta;
            const bool gauss = mu > 0.47f;
            const float den = sqrtf(fmaf(mu, mu, 4.0f)) - mu;
            const float theta = 0.5f * den;
            const float inv_theta = 2.0f / den;
            float zval = 0.0f;
            int32_t att = -1;
            bool done = !active;
            for (uint32_t round = 0; __ballot(!done) != 0ull; ++round) {
                if (!done) {
                    const Words4 w = draw_words(seed, row, kk, kTagZ, round, cid);
                    float ta, tb;
                    bool aa, ab;
                    tn_candidate(mu, gauss, theta, inv_theta, u01f(w.w0), u01f(w.w1), ta, aa);
                    tn_candidate(mu, gauss, theta, inv_theta, u01f(w.w2), u01f(w.w3), tb, ab);
                    if (aa) {
                        zval = ys * ta;
                        att = (int32_t)(2 * round);
                        done = true;
                    } else if (ab) {
                        zval = ys * tb;
                        att = (int32_t)(2 * round + 1);
                        done = true;
                    } else if (round + 1 >= kMaxRounds) {
                        zval = __builtin_nanf("");
                        done = true;
                        capped = true;
                    }
                }
            }
            if (active) {
                maxatt = max(maxatt, (uint32_t)(att + 1));
                if (zdbg) {
                    zdbg[row] = zval;
                    adbg[row] = att | (gauss ? (1 << 30) : 0);
                }
            }
            zl[mrow * kMcChains + n] = zval;
            __syncthreads();

            // X^T z for the 16 chains: B = z of rows 4 q .. 4 q + 3, chain n
            Bf16x4 zhi, zlo;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                uint32_t h, l;
                split_bf16(zl[(4 * q + r) * kMcChains + n], h, l);
                zhi[r] = (short)h;
                zlo[r] = (short)l;
            }
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    db[s][h] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(tt[s][h], zhi, db[s][h], 0, 0, 0);
                    db[s][h] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(tt[s][h], zlo, db[s][h], 0, 0, 0);
                }
        }
        flush();
        if (threadIdx.x == 0) *slot = next;
        __syncthreads();
        u = *slot;
        __syncthreads();
    }
    if (!wrote) flush();  // no unit: the partial is zero

    // per-chain statistics: lanes n, n + 16, n + 32, n + 48 share chain n
    uint32_t mx = maxatt;
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, 16));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, 32));
    const unsigned long long capmask = __ballot(capped);
    const bool anycap = ((capmask >> n) | (capmask >> (n + 16)) | (capmask >> (n + 32)) | (capmask >> (n + 48))) & 1ull;
    if (live && q == 0) {
        if (mx) atomicMax(&ctrl->max_attempts, mx);
        if (anycap) atomicOr(&ctrl->err, kErrTnCap);
    }

    // This block's partial is complete.  The last of each group of kZGroup
    // blocks adds the group's partials in block order into every chain's X^T z
    // accumulator (float64 atomics, exact on the grid); the last group resets
    // the counters for the next launch.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const uint32_t grp = rank / kZGroup;
    const uint32_t g0 = grp * kZGroup;
    const uint32_t gsize = min((uint32_t)kZGroup, m.gz - g0);
    if (threadIdx.x == 0) *slot = atomicAdd(&m.count[grp], 1u) == gsize - 1 ? 1u : 0u;
    __syncthreads();
    const bool last = *slot != 0u;
    __syncthreads();
    if (!last) return;
    for (uint32_t e = threadIdx.x; e < C * ld; e += kThreads) {
        const uint32_t c = e / ld, col = e % ld;
        double v = 0.0;
        for (uint32_t r = 0; r < gsize; ++r) v += ldc(&m.partial[((size_t)(g0 + r) * kMcChains + c) * m.pstride + col]);
        Args& a = *(Args*)m.chain[c];
        __hip_atomic_fetch_add(&a.bsum[col], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0) {
        __hip_atomic_store(&m.count[grp], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (atomicAdd(&m.count[m.zgroups], 1u) == m.zgroups - 1) {
            // every block has left its claim loop
            __hip_atomic_store(&m.count[m.zgroups], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(unit_next, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace hsp
