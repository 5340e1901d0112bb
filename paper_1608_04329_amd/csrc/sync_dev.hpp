// Cross-block ordering inside the sweep kernel (agent scope).
//
// One thread of a block fences for the whole block: every wave first waits
// for its own stores (s_waitcnt) and the block meets at a barrier; then the
// thread writes this XCD's L2 back before it signals (release), or, having
// seen a signal, invalidates the caches before the barrier that lets the
// block's waves read (acquire).  The write-back and the invalidate are memory
// operations of their own: the thread waits for each to complete, so the
// signal cannot overtake the write-back and the other waves' loads cannot
// overtake the invalidate.
#pragma once

namespace hsp {

__device__ __forceinline__ void fence_release() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
}

__device__ __forceinline__ void fence_acquire() {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
}

}  // namespace hsp
