// Device helpers shared by the HIP sources of libuavq.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uavq_kargs.h"

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

// Acceptance cuts of four sites: for each, the least d >= 1 whose table entry thr(d) is
// <= u, so that a flip with energy change dE is accepted exactly when dE < cut
// (dE <= 0 always; 0 < dE < dcut iff u < thr(dE); thr(d) = 0 from dcut on).
// The continuous threshold 2^32 exp(-d/T) drops to u at d = T ln 2 (32 -
// log2 u); a guess half a step below that (e0 = 32 T ln 2 - 1/2) is the cut or
// one short of it, which the entries d-1, d, d+1 settle.  Otherwise (never
// seen: the guess is good to far better than half a step; or u = 2^32 - 1)
// the table is walked.  The result depends on the table alone.  The LDS row
// must hold valid entries up to index dcut + 1.
__device__ __forceinline__ void accept_cuts(const uint4 &u4, float tl2, float e0, float dm1, int dcut,
                                            const uint32_t *thr, int &cut0, int &cut1, int &cut2, int &cut3) {
    const uint32_t u[4] = {u4.x, u4.y, u4.z, u4.w};
    int d[4], cut[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const float e = fmaf(-tl2, __builtin_amdgcn_logf((float)u[i]), e0);   // u = 0: +inf
        d[i] = (int)__builtin_amdgcn_fmed3f(e, 0.0f, dm1) + 1;                // 1..dcut
    }
    // all twelve entries are read unconditionally, so the reads issue together
    uint32_t tm[4], t0[4], t1[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        tm[i] = thr[d[i] - 1];
        t0[i] = thr[d[i]];
        t1[i] = thr[d[i] + 1];
    }
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        cut[i] = d[i] + (t0[i] > u[i] ? 1 : 0);
        ok = ok & (tm[i] > u[i]) & (t1[i] <= u[i]);
    }
    if (ballot64(!ok)) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            int c = cut[i];
            while (c < dcut && thr[c] > u[i]) c++;
            while (c > 1 && thr[c - 1] <= u[i]) c--;
            cut[i] = c;
        }
    }
    cut0 = cut[0];
    cut1 = cut[1];
    cut2 = cut[2];
    cut3 = cut[3];
}

// Philox words of one lane's block of four steps and their exact cuts, packed
// as four uint16.  Out of line: the m <= 64 producer/consumer sweep takes it
// only when no producer made the cuts, and the chunked walks call it from
// many places (one copy instead of one per call site).
static __device__ __attribute__((noinline)) uint2 draw_cuts(uint32_t cbase, uint32_t s, uint32_t r, uint32_t inst, uint32_t seed,
                                                     float tl2, float e0, float dm1, int dcut, const uint32_t *thr) {
    const uint4 u4 = philox(make_uint4(cbase, s, r, inst), seed, 0u);
    int c0, c1, c2, c3;
    accept_cuts(u4, tl2, e0, dm1, dcut, thr, c0, c1, c2, c3);
    return make_uint2((uint32_t)c0 | ((uint32_t)c1 << 16), (uint32_t)c2 | ((uint32_t)c3 << 16));
}

// Work-item loop: one item per block, or (persistent mode) items pulled in
// order from a counter until the class is exhausted.
__device__ __forceinline__ int next_item(const KArgs &a, int iter) {
    __shared__ int s_item;
    if (!a.queue) return iter == 0 ? a.item_base + (int)blockIdx.x : -1;
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(a.queue, 1);
    __syncthreads();
    const int k = s_item;
    return k < a.queue_n ? a.item_base + k : -1;
}

}  // namespace uavq
