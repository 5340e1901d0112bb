// One Gibbs sweep as one kernel launch.
//
// The grid has two roles.  Blocks [0, gp) form the p-side group: lambda^-2,
// tau^-2, nu^-1, xi^-1 and the Cholesky factorisation of Q need only the
// previous sweep, so they run while blocks [gp, gp + gz) stream X through the
// z pass (z | beta and the partial sums of X^T z).  The group then waits for
// the z pass, reduces X^T z and draws beta.  This is the schedule of
// Section 5 -- (i) z in parallel with lambda, then tau; (ii) beta with nu and
// xi -- inside a single launch, so a sweep costs one graph node and the
// p-side work hides under the bandwidth-bound pass over X.
//
// The group blocks come first in the grid: they are dispatched before any
// z-pass block and stay resident, so their barriers only ever wait on
// blocks that are running.  The z-pass blocks never wait on anything.
#include <algorithm>
#include <utility>

#include "mc_dev.hpp"
#include "pside_dev.hpp"
#include "zpass_dev.hpp"

namespace hsp {
namespace {

// The launch's description lives in device memory (read through the scalar
// cache as needed) rather than in kernel arguments, which would otherwise stay
// pinned in scalar registers for the whole kernel.
// A launch may serve several independent chains (a batch): block b belongs
// to chain chain_of_block[b] (chain 0 for all when the map is null) and runs
// that chain's role at position b - block0 of its blocks, or, marked with
// kWorkerBit, is a worker of the pack's shared z queue.
template <int XT, int KC, int R, bool WIDE>
__device__ __forceinline__ void run_block(Args& a, double* lds) {
    uint32_t b = blockIdx.x - a.block0;
    const uint32_t k = a.ctrl->sweep + 1u;
    if (a.idle) {
        if (b == a.idle) return;
        if (b > a.idle) --b;
    }
    if (b < a.gp) pside_role(a, b, k, lds);
    else zpass_role<XT, KC, R, WIDE>(a, b - a.gp, a.gz, k, lds);
}

// KC: 16-byte chunks per lane of a wave (of the whole row, or with WIDE of
// the wave's quarter of it); R: rows per tile.
template <int XT, int KC, int R, bool WIDE>
__global__ __launch_bounds__(kThreads, 2) void sweep_kernel(const SweepArgs* const* __restrict__ args,
                                                            const uint16_t* __restrict__ chain_of_block) {
    __shared__ double lds[kLdsDoubles];
    const uint32_t c = chain_of_block ? chain_of_block[blockIdx.x] : 0u;
    if constexpr (!WIDE) {
        if (c & kWorkerBit) {
            zqueue_role<XT, KC, R>(args, c & ~(uint32_t)kWorkerBit, lds);
            return;
        }
    }
    run_block<XT, KC, R, WIDE>(*(Args*)args[c], lds);
}



// The multi-chain z pass for chains sharing one bfloat16 design (KS
// 32-column steps per wave); no block waits for another.
template <int KS>
__global__ __launch_bounds__(kThreads, 2) void mc_zpass_kernel(const McArgs* __restrict__ mc) {
    __shared__ double lds[kMcLdsDoubles];
    McView& m = *(McView*)mc;
    mc_role<KS>(m, blockIdx.x, lds);
}

using KernelFn = void (*)(const SweepArgs* const*, const uint16_t*);

template <int XT, int... KCs>
KernelFn pick(int kc, std::integer_sequence<int, KCs...>) {
    KernelFn f = nullptr;
    ((kc == KCs + 1 ? (f = &sweep_kernel<XT, KCs + 1, rows_for(XT, KCs + 1), false>, 0) : 0), ...);
    return f;
}

// wide rows: kcw chunks per lane of each wave's quarter
template <int XT, int... KCs>
KernelFn pick_wide(int kcw, std::integer_sequence<int, KCs...>) {
    KernelFn f = nullptr;
    ((kcw == KCs + 1 ? (f = &sweep_kernel<XT, KCs + 1, rows_for(XT, 4 * (KCs + 1)), true>, 0) : 0), ...);
    return f;
}

KernelFn kernel_for(int xtype, int chunks) {
    if (!wide_chunks(xtype, chunks)) {
        if (xtype == 0) return pick<0>(chunks, std::make_integer_sequence<int, 6>{});
        return pick<1>(chunks, std::make_integer_sequence<int, 2>{});
    }
    const int kcw = (chunks + 3) / 4;
    if (xtype == 0) return pick_wide<0>(kcw, std::make_integer_sequence<int, kMaxP / (kWave * 4 * 4)>{});
    return pick_wide<1>(kcw, std::make_integer_sequence<int, kMaxP / (kWave * 8 * 4)>{});
}

}  // namespace

uint32_t max_group(const XLayout& x, int capacity) {
    const uint32_t nt = (x.p + kTile - 1) / kTile;
    uint32_t gp = x.p <= (uint32_t)kSmallP ? 1u : nt * (nt + 1) / 2;
    // the factorisation's tile tasks (each ~6 us on one block) against the
    // pass over X (~6 TB/s) on the other three quarters of the device
    double tasks = 0.0;
    for (uint32_t k = 0; x.p > (uint32_t)kSmallP && k < nt; ++k) {
        const double m = nt - k - 1;
        tasks += 1.0 + m + m * (m + 1.0) / 2.0 + (with_inverse(nt) ? k + m * (k + 1.0) : 0.0);
    }
    const double z_us = (double)x.N * x.ld * (x.xtype == 0 ? 4 : 2) / 6.0e6;
    const bool factor_bound = tasks * 6.0 / (kMaxGroup - 1) > z_us;
    if (x.p <= kLargeP && !factor_bound) {
        // the factorisation hides under the z pass: a quarter of the device at most
        if (gp > (uint32_t)kMaxGroup) gp = kMaxGroup;
        if (gp > (uint32_t)capacity / 4) gp = capacity / 4 > 0 ? capacity / 4 : 1;
    } else {
        // the factorisation outweighs the pass over X: three quarters
        const uint32_t cap = (uint32_t)capacity * 3 / 4;
        if (gp > cap) gp = cap > 0 ? cap : 1;
    }
    return gp;
}

hipError_t sweep_plan(const XLayout& x, int num_cus, SweepPlan* plan, uint32_t gp_req) {
    const int vec = x.xtype == 0 ? 4 : 8;
    plan->chunks = (int)((x.ld + kWave * vec - 1) / (kWave * vec));
    plan->rows = rows_for(x.xtype, plan->chunks);
    const bool wide = wide_chunks(x.xtype, plan->chunks);
    KernelFn f = kernel_for(x.xtype, plan->chunks);
    if (!f) return hipErrorInvalidValue;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(f),
                                                                kThreads, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    plan->capacity = per_cu * num_cus;
    plan->cus = (uint32_t)num_cus;
    uint32_t gp = max_group(x, plan->capacity);
    if (gp_req > 0 && gp_req < gp) gp = gp_req;
    plan->gp = gp;
    const uint64_t tiles = (x.N + plan->rows - 1) / plan->rows;
    // a wave takes a tile (a block, for wide rows)
    uint64_t gz = wide ? tiles : (tiles + kWPB - 1) / kWPB;
    const uint64_t room = (uint64_t)plan->capacity - gp;
    if (gz > room) gz = room;
    if (gz < 1) gz = 1;
    plan->gz = (uint32_t)gz;
    return hipSuccess;
}

// Blocks b and b + (compute units) of a full grid share a compute unit (the
// dispatcher deals blocks out to the units in order, twice round).  When a
// launch fills the device at two blocks per unit, block 0 (the p-side's
// critical chain) would share its unit with a z-pass block; that block is
// left idle instead, and the z pass takes one block fewer: the chain then
// has its unit to itself (N = 1e6, p = 1000 bfloat16: 0.415 -> 0.402 ms per
// sweep; float32, bound by its z pass, unchanged).
void sweep_finish_args(SweepArgs* a, const SweepPlan& plan) {
    a->gp = plan.gp;
    a->gz = (a->mode & kModeZ) ? plan.gz : 0u;
    a->idle = 0u;
    if (a->gp > 0u && a->gz > plan.cus && plan.capacity == 2 * (int)plan.cus &&
        a->gp + a->gz == (uint32_t)plan.capacity) {
        a->gz -= 1u;
        a->idle = plan.cus;
    }
    a->zgroups = (a->gz + kZGroup - 1) / kZGroup;
    a->z_static_pct = plan.static_pct;
    a->z_unit = plan.unit;
}

hipError_t sweep_launch(const SweepArgs& host, const SweepArgs* const* table, const SweepPlan& plan,
                        hipStream_t st) {
    KernelFn f = kernel_for(host.x.xtype, plan.chunks);
    if (!f) return hipErrorInvalidValue;
    const uint16_t* none = nullptr;
    void* args[] = {&table, &none};
    return hipLaunchKernel(reinterpret_cast<const void*>(f), dim3(host.gp + host.gz + (host.idle ? 1u : 0u)),
                           dim3(kThreads),
                           args, 0, st);
}

int pack_capacity(int xtype, int chunks, int num_cus) {
    KernelFn f = kernel_for(xtype, chunks);
    int per_cu = 0;
    if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(f),
                                                           kThreads, 0) != hipSuccess)
        return 0;
    return per_cu * num_cus;
}

hipError_t mc_launch(const McArgs* mc, uint32_t ld, uint32_t gz, hipStream_t st) {
    if (ld > kMcMaxLd) return hipErrorInvalidValue;
    void* args[] = {&mc};
    const void* f = mc_steps(ld) == 4u ? reinterpret_cast<const void*>(&mc_zpass_kernel<4>)
                                       : reinterpret_cast<const void*>(&mc_zpass_kernel<kMcKs>);
    return hipLaunchKernel(f, dim3(gz), dim3(kThreads), args, 0, st);
}

hipError_t pack_launch(int xtype, int chunks, const SweepArgs* const* table, const uint16_t* chain_of_block,
                       uint32_t blocks, hipStream_t st) {
    KernelFn f = kernel_for(xtype, chunks);
    if (!f) return hipErrorInvalidValue;
    void* args[] = {&table, &chain_of_block};
    return hipLaunchKernel(reinterpret_cast<const void*>(f), dim3(blocks), dim3(kThreads), args, 0, st);
}

}  // namespace hsp
