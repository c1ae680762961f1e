// Device side of a batched launch (SlotBatch): copy blockIdx.z of the grid
// works on the buffers of slot z, at byte offset off[z] from the launch's
// pointers; a null pointer stays null.
#pragma once

#include <type_traits>

#include "tng_internal.hpp"

namespace tng {

// Byte-pointer arithmetic (not an integer round trip), so the compiler keeps
// the kernel argument's global address space and emits global, not flat,
// memory instructions.
template <class P>
__device__ __forceinline__ P* at_slot(P* p, long long off) {
    using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
    return p == nullptr ? p : reinterpret_cast<P*>(reinterpret_cast<B*>(p) + off);
}

__device__ __forceinline__ long long slot_off(const SlotBatch& sb) { return sb.off[blockIdx.z]; }

// vector count (or table index) of this copy: the per-slot one when given
__device__ __forceinline__ int slot_count(const SlotBatch& sb, int n) {
    return sb.has_cnt ? sb.cnt[blockIdx.z] : n;
}

}  // namespace tng
