// Device helpers shared by the HIP sources of libuavq.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uavq_internal.h"

#define UAVQ_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::uavq::set_error(UAVQ_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

namespace uavq {

static __host__ __device__ inline size_t al16(size_t v) { return (v + 15) & ~(size_t)15; }

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 products
// with the published multipliers, the key bumped by the Weyl constants.
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; i++) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;   // one v_mad_u64_u32 each
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Read-only plan data read at wave-uniform addresses: through the constant
// address space so that it is fetched with scalar loads (no vector-memory
// wait that would also wait for in-flight vector loads).
typedef __attribute__((address_space(4))) const int32_t const_i32;
__device__ __forceinline__ int32_t uniform_load(const int32_t *p, int i) { return ((const_i32 *)p)[i]; }

}  // namespace uavq
