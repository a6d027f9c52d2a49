// Kernels of the block-tested chunked sweep for two to four chunks per lane
// (64 < m <= 256); the sweep itself is chunk_item in uavq_chunk.h.
#include "uavq_chunk.h"

namespace uavq {

template <int NJ, bool STOP>
__global__ __launch_bounds__(1024) void k_sweep_chunk(KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int iter = 0;; iter++) {
        const int itx = next_item(a, iter);
        if (itx < 0) break;
        chunk_item<NJ, STOP>(a, itx, smem);
    }
}

// Four chunks (192 < m <= 256, fields up to 16x16): 32 mask words per lane, so at most four waves per block and
// two per SIMD, as for the generic kernel of that class.
template <bool STOP>
__global__ __launch_bounds__(64 * kWideMaxWaves) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_sweep_chunk4(
    KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int iter = 0;; iter++) {
        const int itx = next_item(a, iter);
        if (itx < 0) break;
        chunk_item<4, STOP>(a, itx, smem);
    }
}

const void *chunk_sweep_kernel(int nj, bool stop) {
    if (nj == 2) return stop ? (const void *)k_sweep_chunk<2, true> : (const void *)k_sweep_chunk<2, false>;
    if (nj == 3) return stop ? (const void *)k_sweep_chunk<3, true> : (const void *)k_sweep_chunk<3, false>;
    if (nj == 4) return stop ? (const void *)k_sweep_chunk4<true> : (const void *)k_sweep_chunk4<false>;
    return nullptr;
}

}  // namespace uavq
