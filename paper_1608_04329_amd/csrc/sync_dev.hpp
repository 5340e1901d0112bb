// Hand-offs between blocks inside the sweep kernel.
//
// Data that one block hands to another within a launch (factorisation tiles,
// partial sums of X^T z, lambda^-2, the noise and y vectors) moves only
// through device-coherent loads and stores (relaxed atomics at agent scope,
// which bypass the caches that are not coherent across XCDs).  A hand-off
// then needs no cache maintenance: the writer's waves wait for their own
// stores (s_waitcnt) and meet at a barrier before one thread signals (a
// counter or a tile version), and the reader loads only after it has seen
// the signal.  Agent-scope fences would instead write back or invalidate a
// whole XCD's L2 (and must then also be waited for), stalling the z pass
// that streams through the same L2.
#pragma once

namespace hsp {

__device__ __forceinline__ double ldc(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stc(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace hsp
