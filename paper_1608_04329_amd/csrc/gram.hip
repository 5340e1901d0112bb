// One-time work at creation: the column scales of X, X packed into the
// library layout, input validation, and G = X^T X in float64 (Section 5,
// beta step i).  Also the device Philox test hook and the read-ceiling probe.
#include <mutex>

#include "hsp_internal.hpp"
#include "philox.hpp"

namespace hsp {
namespace {

__device__ __forceinline__ float load_x(const XLayout& x, size_t row, uint32_t col) {
    if (x.xtype == 0) return static_cast<const float*>(x.X)[row * x.ld + col];
    const uint32_t bits = (uint32_t) static_cast<const uint16_t*>(x.X)[row * x.ld + col] << 16;
    return __uint_as_float(bits);
}

// float32 -> bfloat16, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Column maxima of |x|: block (bx, by) scans rows [bx R, bx R + R) of the 256
// columns at by * 256, one column per thread (a row's columns are adjacent
// threads, so every load instruction reads one contiguous row segment), and
// merges its maximum into out[col] by an atomic maximum on the bit pattern
// (non-negative floats order as unsigned integers; NaN sorts above infinity).
constexpr uint32_t kColmaxRows = 512;
__global__ __launch_bounds__(256) void colmax_kernel(const float* __restrict__ src, uint32_t N, uint32_t p,
                                                     uint32_t* __restrict__ out) {
    const uint32_t col = blockIdx.y * 256u + threadIdx.x;
    if (col >= p) return;
    const size_t r0 = (size_t)blockIdx.x * kColmaxRows;
    const size_t r1 = min((size_t)N, r0 + kColmaxRows);
    uint32_t m = 0;
    for (size_t r = r0; r < r1; ++r) m = max(m, __float_as_uint(src[r * p + col]) & 0x7FFFFFFFu);
    atomicMax(&out[col], m);
}

// The library's copy: column j multiplied by 2^-e[j] (exact), rounded to
// bfloat16 if asked (rounding commutes with the power-of-two scale).  Each
// element is read and written by the same thread, so src may alias dst when
// the two layouts coincide.
__global__ void pack_kernel(const float* src, XLayout dst, const int32_t* __restrict__ e) {
    const size_t n = (size_t)dst.N * dst.ld;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t row = idx / dst.ld;
        const uint32_t col = (uint32_t)(idx % dst.ld);
        const float v = col < dst.p ? ldexpf(src[row * dst.p + col], -e[col]) : 0.0f;
        if (dst.xtype == 0) const_cast<float*>(static_cast<const float*>(dst.X))[idx] = v;
        else const_cast<uint16_t*>(static_cast<const uint16_t*>(dst.X))[idx] = to_bf16(v);
    }
}

__global__ void validate_kernel(XLayout x, const uint8_t* __restrict__ y, Ctrl* ctrl) {
    const size_t n = (size_t)x.N * x.ld;
    bool bad = false;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * blockDim.x) {
        if (!isfinite(load_x(x, idx / x.ld, (uint32_t)(idx % x.ld)))) bad = true;
    }
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < x.N;
         i += (size_t)gridDim.x * blockDim.x)
        if (y[i] > 1) bad = true;
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&ctrl->err, kErrInput);
}

// ---- G = X^T X on the FP64 matrix cores ---------------------------------------
// The upper triangle of G is cut into 64 x 64 tiles (ti <= tj, "pairs") and
// the rows of X into splits.  Block (pair, split) stages 64 rows of X's
// column tiles ti and tj in LDS as float64 (exact) and accumulates
// X_ti^T X_tj with v_mfma_f64_16x16x4f64: wave w owns the 32 x 32 quadrant
// at (32 (w / 2), 32 (w % 2)) as 2 x 2 blocks of 16 x 16; lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16], i.e. rows of the stage are the
// contraction index, and holds D[l / 16 + 4 r][l % 16] in its r-th result.
// The next stage's loads are issued before the current stage's products.
// Every split writes its partial tile; a second kernel sums the splits of
// each entry in split order, so G does not depend on timing.
constexpr int kGT = 64;
typedef double GAcc __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void pair_of(uint32_t pair, uint32_t nt, uint32_t& ti, uint32_t& tj) {
    uint32_t r = 0, idx = pair;
    while (idx >= nt - r) { idx -= nt - r; ++r; }
    ti = r;
    tj = r + idx;
}

// Pairs [pair0, pair0 + gridDim.x) over the row splits of x, which are the
// splits split0, split0 + 1, ... of the whole design (x may be a chunk of its
// rows); work holds gridDim.x tiles per split, split-major.
__global__ __launch_bounds__(256) void gram_tile_kernel(XLayout x, double* __restrict__ work, uint32_t nt,
                                                        uint32_t pair0, uint32_t rows_per_split, uint32_t split0) {
    __shared__ double S[kGT][kGT + 2];
    __shared__ double T[kGT][kGT + 2];
    uint32_t ti, tj;
    pair_of(pair0 + blockIdx.x, nt, ti, tj);
    const size_t r_begin = (size_t)blockIdx.y * rows_per_split;
    const size_t r_end = min((size_t)x.N, r_begin + rows_per_split);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kr = lane >> 4, cc = lane & 15;
    const int i0 = 32 * (wave >> 1), j0 = 32 * (wave & 1);
    // staging: thread t loads column t % 64 of stage rows t / 64 + 4 q
    const int c = threadIdx.x & (kGT - 1), rb = threadIdx.x >> 6;
    const uint32_t ca = ti * kGT + c, cb = tj * kGT + c;
    const bool diag = ti == tj;
    GAcc acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = GAcc{0.0, 0.0, 0.0, 0.0};
    double va[16], vb[16];
    auto fetch = [&](size_t r0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const size_t row = r0 + rb + 4 * q;
            const bool in = row < r_end;
            va[q] = (in && ca < x.p) ? (double)load_x(x, row, ca) : 0.0;
            vb[q] = (!diag && in && cb < x.p) ? (double)load_x(x, row, cb) : 0.0;
        }
    };
    if (r_begin < r_end) fetch(r_begin);
    for (size_t r0 = r_begin; r0 < r_end; r0 += kGT) {
        __syncthreads();  // the previous stage's products have read S and T
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            S[rb + 4 * q][c] = va[q];
            if (!diag) T[rb + 4 * q][c] = vb[q];
        }
        __syncthreads();
        if (r0 + kGT < r_end) fetch(r0 + kGT);
        const double(*B)[kGT + 2] = diag ? S : T;
#pragma unroll 4
        for (int q0 = 0; q0 < kGT; q0 += 4) {
            const double a0 = S[q0 + kr][i0 + cc], a1 = S[q0 + kr][i0 + 16 + cc];
            const double b0 = B[q0 + kr][j0 + cc], b1 = B[q0 + kr][j0 + 16 + cc];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
    double* out = work + ((size_t)(split0 + blockIdx.y) * gridDim.x + blockIdx.x) * (kGT * kGT);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(i0 + 16 * bi + kr + 4 * r) * kGT + j0 + 16 * bj + cc] = acc[bi][bj][r];
}

// G from the partial tiles of pairs [pair0, pair0 + npc), summed over the
// splits in order, mirrored, and unscaled by 2^(e_i + e_j) (exact) if e.
__global__ void gram_reduce_kernel(const double* __restrict__ work, uint32_t nsplit, uint32_t npc,
                                   uint32_t pair0, uint32_t nt, uint32_t p, const int32_t* __restrict__ e,
                                   double* __restrict__ G) {
    const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (idx >= (size_t)npc * kGT * kGT) return;
    const uint32_t pc = (uint32_t)(idx / (kGT * kGT)), local = (uint32_t)(idx % (kGT * kGT));
    uint32_t ti, tj;
    pair_of(pair0 + pc, nt, ti, tj);
    const uint32_t i = ti * kGT + local / kGT, j = tj * kGT + local % kGT;
    if (i >= p || j >= p || (ti == tj && j < i)) return;
    double s = 0.0;
    for (uint32_t sp = 0; sp < nsplit; ++sp) s += work[((size_t)sp * npc + pc) * (kGT * kGT) + local];
    if (e) s = ldexp(s, e[i] + e[j]);
    G[(size_t)i * p + j] = s;
    G[(size_t)j * p + i] = s;
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

__global__ void pad_gram_kernel(const double* __restrict__ G, uint32_t p, uint32_t P,
                                double* __restrict__ Gp) {
    const size_t n = (size_t)P * P;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)(e / P), j = (uint32_t)(e % P);
        Gp[e] = (i < p && j < p) ? G[(size_t)i * p + j] : (i == j ? 1.0 : 0.0);
    }
}

}  // namespace

GramGeometry gram_geometry(const XLayout& x, int num_cus, uint64_t max_rows_per_split) {
    GramGeometry g;
    g.nt = (x.p + kGT - 1) / kGT;
    g.npairs = g.nt * (g.nt + 1) / 2;
    const uint64_t want = (uint64_t)num_cus * 4;
    uint64_t ns = (want + g.npairs - 1) / g.npairs;
    const uint64_t max_split = (x.N + kGT - 1) / kGT;
    if (ns > max_split) ns = max_split;
    if (ns < 1) ns = 1;
    uint64_t rps = (x.N + ns - 1) / ns;
    rps = (rps + kGT - 1) / kGT * kGT;
    if (max_rows_per_split >= (uint64_t)kGT && rps > max_rows_per_split) rps = max_rows_per_split / kGT * kGT;
    g.nsplit = (uint32_t)((x.N + rps - 1) / rps);
    g.rows_per_split = (uint32_t)rps;
    return g;
}

size_t gram_work_doubles(const XLayout& x, int num_cus) {
    const GramGeometry g = gram_geometry(x, num_cus);
    return (size_t)g.nsplit * g.npairs * kGT * kGT;
}

hipError_t gram_launch_chunked(const XLayout& x, const int32_t* e, double* G, double* work,
                               size_t work_doubles, int num_cus, hipStream_t st) {
    const GramGeometry g = gram_geometry(x, num_cus);
    const size_t per_pair = (size_t)g.nsplit * kGT * kGT;
    const size_t chunk = std::min<size_t>(g.npairs, work_doubles / per_pair);
    if (chunk < 1) return hipErrorInvalidValue;
    for (uint32_t pair0 = 0; pair0 < g.npairs; pair0 += (uint32_t)chunk) {
        const uint32_t npc = (uint32_t)std::min<size_t>(chunk, g.npairs - pair0);
        hipLaunchKernelGGL(gram_tile_kernel, dim3(npc, g.nsplit), dim3(256), 0, st, x, work, g.nt, pair0,
                           g.rows_per_split, 0u);
        const size_t n = (size_t)npc * kGT * kGT;
        hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           (const double*)work, g.nsplit, npc, pair0, g.nt, x.p, e, G);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

// A fixed device workspace for callers that cannot allocate: gram_scratch()
// returns its device address on the current device (found once per device
// with hipGetSymbolAddress; the array's name is not a device address in host
// code).  Every call on one device shares it.
namespace {
__device__ __align__(256) double scratch[kGramScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t gram_scratch(double** ptr) {
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t gram_pair_doubles(const XLayout& x, int num_cus) {
    return (size_t)gram_geometry(x, num_cus).nsplit * kGT * kGT;
}

hipError_t gram_launch(const XLayout& x, const int32_t* e, double* G, double* work, int num_cus,
                       hipStream_t st) {
    return gram_launch_chunked(x, e, G, work, gram_work_doubles(x, num_cus), num_cus, st);
}

hipError_t gram_chunk_launch(const XLayout& chunk, const GramGeometry& g, uint32_t split0, double* work,
                             hipStream_t st) {
    const uint32_t ns = (chunk.N + g.rows_per_split - 1) / g.rows_per_split;
    if (ns == 0) return hipSuccess;
    if (split0 + ns > g.nsplit) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gram_tile_kernel, dim3(g.npairs, ns), dim3(256), 0, st, chunk, work, g.nt, 0u,
                       g.rows_per_split, split0);
    return hipGetLastError();
}

hipError_t gram_reduce_launch(const double* work, const GramGeometry& g, uint32_t p, const int32_t* e, double* G,
                              hipStream_t st) {
    const size_t n = (size_t)g.npairs * kGT * kGT;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, work, g.nsplit,
                       g.npairs, 0u, g.nt, p, e, G);
    return hipGetLastError();
}

hipError_t pad_gram_launch(const double* G, uint32_t p, uint32_t P, double* Gp, hipStream_t st) {
    hipLaunchKernelGGL(pad_gram_kernel, dim3(1024), dim3(256), 0, st, G, p, P, Gp);
    return hipGetLastError();
}

// key[i] = (2 y_i - 1) sum_j x_ij beta32_j: one wave per row (lanes over
// columns, a wave-wide sum), float32, over the stored column-scaled X.
__global__ __launch_bounds__(256) void row_key_kernel(XLayout x, const float* __restrict__ b32,
                                                      const uint8_t* __restrict__ y, float* __restrict__ key) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t waves = gridDim.x * (blockDim.x / 64u);
    for (uint32_t i = blockIdx.x * (blockDim.x / 64u) + threadIdx.x / 64u; i < x.N; i += waves) {
        float acc = 0.0f;
        for (uint32_t j = lane; j < x.p; j += 64u) acc = fmaf(load_x(x, i, j), b32[j], acc);
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) key[i] = y[i] ? acc : -acc;
    }
}

// Row i of Xo is row perm[i] of X (16-byte vectors; a row is ld elements,
// a multiple of 16 bytes), with y and the original row indices alongside.
__global__ __launch_bounds__(256) void gather_rows_kernel(XLayout x, const uint32_t* __restrict__ perm,
                                                          uint4* __restrict__ Xo, const uint8_t* __restrict__ y,
                                                          uint8_t* __restrict__ yo, const uint32_t* __restrict__ id,
                                                          uint32_t* __restrict__ ido) {
    const size_t vpr = (size_t)x.ld * (x.xtype == 0 ? 4 : 2) / 16;  // 16-byte vectors per row
    const uint4* X = static_cast<const uint4*>(x.X);
    for (uint32_t i = blockIdx.x; i < x.N; i += gridDim.x) {
        const uint32_t src = perm[i];
        for (size_t v = threadIdx.x; v < vpr; v += blockDim.x) Xo[(size_t)i * vpr + v] = X[(size_t)src * vpr + v];
        if (threadIdx.x == 0) {
            yo[i] = y[src];
            ido[i] = id ? id[src] : src;
        }
    }
}

// Read ceiling: stream `bytes` (a multiple of 16) with eight 16-byte
// non-temporal loads in flight per lane, grid-stride, the same kind of load
// as the z pass, and nothing else.
typedef unsigned int RdVec __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void stream_read_kernel(const RdVec* __restrict__ x, size_t n16,
                                                          float* __restrict__ sink) {
    constexpr int kUnroll = 8;
    float s = 0.0f;
    size_t i = (size_t)blockIdx.x * 256 * kUnroll + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * 256 * kUnroll;
    for (; i + 256 * (kUnroll - 1) < n16; i += stride) {
        RdVec v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(x + i + 256 * u);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) s += __uint_as_float(v[u].x ^ v[u].y ^ v[u].z ^ v[u].w);
    }
    for (; i < n16; i += 256) {  // the ragged end, one load at a time
        const RdVec v = __builtin_nontemporal_load(x + i);
        s += __uint_as_float(v.x ^ v.y ^ v.z ^ v.w);
    }
    if (s == -1.0f) sink[0] = s;  // never true for the sums of finite data; keeps the loads
}

hipError_t stream_read_launch(const void* x, size_t bytes, int num_cus, float* sink, hipStream_t st) {
    const size_t n16 = bytes / 16;
    const unsigned blocks = (unsigned)(2 * num_cus);
    hipLaunchKernelGGL(stream_read_kernel, dim3(blocks), dim3(256), 0, st,
                       static_cast<const RdVec*>(x), n16, sink);
    return hipGetLastError();
}

hipError_t row_key_launch(const XLayout& x, const float* beta32, const uint8_t* y, float* key, hipStream_t st) {
    hipLaunchKernelGGL(row_key_kernel, dim3(4096), dim3(256), 0, st, x, beta32, y, key);
    return hipGetLastError();
}

hipError_t gather_rows_launch(const XLayout& x, const uint32_t* perm, void* Xo, const uint8_t* y, uint8_t* yo,
                              const uint32_t* id, uint32_t* ido, hipStream_t st) {
    hipLaunchKernelGGL(gather_rows_kernel, dim3(8192), dim3(256), 0, st, x, perm, static_cast<uint4*>(Xo), y, yo,
                       id, ido);
    return hipGetLastError();
}

hipError_t philox_test_launch(uint64_t seed, const uint32_t* ctr, uint32_t n, uint32_t* out,
                              hipStream_t st) {
    hipLaunchKernelGGL(philox_test_kernel, dim3((n + 255) / 256), dim3(256), 0, st, seed, ctr, n, out);
    return hipGetLastError();
}

hipError_t colmax_launch(const float* src, uint32_t N, uint32_t p, uint32_t* colmax_bits, hipStream_t st) {
    const dim3 grid((N + kColmaxRows - 1) / kColmaxRows, (p + 255) / 256);
    hipLaunchKernelGGL(colmax_kernel, grid, dim3(256), 0, st, src, N, p, colmax_bits);
    return hipGetLastError();
}

hipError_t pack_x_launch(const float* src, const XLayout& dst, const int32_t* e, hipStream_t st) {
    hipLaunchKernelGGL(pack_kernel, dim3(4096), dim3(256), 0, st, src, dst, e);
    return hipGetLastError();
}

hipError_t validate_launch(const XLayout& x, const uint8_t* y, Ctrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL(validate_kernel, dim3(4096), dim3(256), 0, st, x, y, ctrl);
    return hipGetLastError();
}

}  // namespace hsp
