// One-time work at creation: pack X into the library layout, validate the
// inputs, and form G = X^T X in float64 (Section 5, beta step i).  Also the
// device Philox test hook.
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

__global__ void pack_kernel(const float* __restrict__ src, XLayout dst) {
    const size_t n = (size_t)dst.N * dst.ld;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t row = idx / dst.ld;
        const uint32_t col = (uint32_t)(idx % dst.ld);
        const float v = col < dst.p ? src[row * dst.p + col] : 0.0f;
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

constexpr int kGT = 64;   // Gram tile
constexpr int kGK = 32;   // rows per LDS stage

__device__ __forceinline__ void pair_of(uint32_t pair, uint32_t nt, uint32_t& ti, uint32_t& tj) {
    uint32_t r = 0, idx = pair;
    while (idx >= nt - r) { idx -= nt - r; ++r; }
    ti = r;
    tj = r + idx;
}

// Partial Gram tile (ti, tj), ti <= tj, over the row range of split blockIdx.y.
__global__ __launch_bounds__(256) void gram_tile_kernel(XLayout x, double* __restrict__ work,
                                                        uint32_t nt, uint32_t rows_per_split) {
    __shared__ double As[kGK][kGT + 1];
    __shared__ double Bs[kGK][kGT + 1];
    uint32_t ti, tj;
    pair_of(blockIdx.x, nt, ti, tj);
    const uint32_t npairs = gridDim.x;
    const size_t r_begin = (size_t)blockIdx.y * rows_per_split;
    const size_t r_end = min((size_t)x.N, r_begin + rows_per_split);
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    double acc[4][4] = {};
    for (size_t r0 = r_begin; r0 < r_end; r0 += kGK) {
        for (int e = tid; e < kGK * kGT; e += 256) {
            const int q = e / kGT, c = e % kGT;
            const size_t row = r0 + q;
            const uint32_t ca = ti * kGT + c, cb = tj * kGT + c;
            As[q][c] = (row < r_end && ca < x.p) ? (double)load_x(x, row, ca) : 0.0;
            Bs[q][c] = (row < r_end && cb < x.p) ? (double)load_x(x, row, cb) : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int q = 0; q < kGK; ++q) {
            double a[4], b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                a[t] = As[q][ty * 4 + t];
                b[t] = Bs[q][tx * 4 + t];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[t][u] += a[t] * b[u];
        }
        __syncthreads();
    }
    double* out = work + ((size_t)blockIdx.y * npairs + blockIdx.x) * (kGT * kGT);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) out[(ty * 4 + t) * kGT + tx * 4 + u] = acc[t][u];
}

// G from the partial tiles, summed over the splits in order, mirrored.
__global__ void gram_reduce_kernel(const double* __restrict__ work, uint32_t nsplit,
                                   uint32_t npairs, uint32_t nt, uint32_t p, double* __restrict__ G) {
    const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (e >= (size_t)npairs * kGT * kGT) return;
    const uint32_t pair = (uint32_t)(e / (kGT * kGT)), local = (uint32_t)(e % (kGT * kGT));
    uint32_t ti, tj;
    pair_of(pair, nt, ti, tj);
    const uint32_t i = ti * kGT + local / kGT, j = tj * kGT + local % kGT;
    if (i >= p || j >= p || (ti == tj && j < i)) return;
    double s = 0.0;
    for (uint32_t sp = 0; sp < nsplit; ++sp) s += work[((size_t)sp * npairs + pair) * (kGT * kGT) + local];
    G[(size_t)i * p + j] = s;
    G[(size_t)j * p + i] = s;
}

void gram_geometry(const XLayout& x, int num_cus, uint32_t& nt, uint32_t& npairs, uint32_t& nsplit,
                   uint32_t& rows_per_split) {
    nt = (x.p + kGT - 1) / kGT;
    npairs = nt * (nt + 1) / 2;
    const uint64_t want = (uint64_t)num_cus * 4;
    uint64_t ns = (want + npairs - 1) / npairs;
    const uint64_t max_split = (x.N + kGK - 1) / kGK;
    if (ns > max_split) ns = max_split;
    if (ns < 1) ns = 1;
    uint64_t rps = (x.N + ns - 1) / ns;
    rps = (rps + kGK - 1) / kGK * kGK;
    nsplit = (uint32_t)((x.N + rps - 1) / rps);
    rows_per_split = (uint32_t)rps;
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

hipError_t pad_gram_launch(const double* G, uint32_t p, uint32_t P, double* Gp, hipStream_t st) {
    hipLaunchKernelGGL(pad_gram_kernel, dim3(1024), dim3(256), 0, st, G, p, P, Gp);
    return hipGetLastError();
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

hipError_t philox_test_launch(uint64_t seed, const uint32_t* ctr, uint32_t n, uint32_t* out,
                              hipStream_t st) {
    hipLaunchKernelGGL(philox_test_kernel, dim3((n + 255) / 256), dim3(256), 0, st, seed, ctr, n, out);
    return hipGetLastError();
}

hipError_t pack_x_launch(const float* src, const XLayout& dst, hipStream_t st) {
    hipLaunchKernelGGL(pack_kernel, dim3(4096), dim3(256), 0, st, src, dst);
    return hipGetLastError();
}

hipError_t validate_launch(const XLayout& x, const uint8_t* y, Ctrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL(validate_kernel, dim3(4096), dim3(256), 0, st, x, y, ctrl);
    return hipGetLastError();
}

size_t gram_work_doubles(const XLayout& x, int num_cus) {
    uint32_t nt, npairs, nsplit, rps;
    gram_geometry(x, num_cus, nt, npairs, nsplit, rps);
    return (size_t)nsplit * npairs * kGT * kGT;
}

hipError_t gram_launch(const XLayout& x, double* G, double* work, int num_cus, hipStream_t st) {
    uint32_t nt, npairs, nsplit, rps;
    gram_geometry(x, num_cus, nt, npairs, nsplit, rps);
    hipLaunchKernelGGL(gram_tile_kernel, dim3(npairs, nsplit), dim3(256), 0, st, x, work, nt, rps);
    const size_t n = (size_t)npairs * kGT * kGT;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (const double*)work, nsplit, npairs, nt, x.p, G);
    return hipGetLastError();
}

}  // namespace hsp
