// Kernels of the block-tested chunked sweep for five and six chunks per lane
// (256 < m <= 384, fields up to 19x19; the sweep itself is chunk_item in
// uavq_chunk.h).  Up to 72 mask words per lane: one wave per SIMD, at most
// four per block, as for the generic kernels of these classes.
#include "uavq_chunk.h"

namespace uavq {

template <int NJ>
__global__ __launch_bounds__(64 * kWideMaxWaves) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_sweep_chunk_wide(
    KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int iter = 0;; iter++) {
        const int itx = next_item(a, iter);
        if (itx < 0) break;
        chunk_item<NJ, false>(a, itx, smem);
    }
}

// One build per class, and none stops frozen replicas: with UAVQ_STOP_FROZEN
// these classes sweep to the end, which gives the same outputs.
const void *chunk_sweep_wide_kernel(int nj, bool stop) {
    (void)stop;
    if (nj == 5) return (const void *)k_sweep_chunk_wide<5>;
    if (nj == 6) return (const void *)k_sweep_chunk_wide<6>;
    return nullptr;
}

}  // namespace uavq
