// Kernels of the block-tested chunked sweep for chunk classes 7..9 (m <= 576,
// fields up to 24x24) and every field whose travel costs exceed a byte: the
// cost matrix is read as 16-bit entries from global memory (it stays in each
// XCD's L2), LDS holds only the acceptance-table row.  One wave per SIMD, at
// most four per block.
#include "uavq_chunk.h"

namespace uavq {

template <int NJ>
__global__ __launch_bounds__(64 * kWideMaxWaves) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_sweep_chunk_big(
    KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int iter = 0;; iter++) {
        const int itx = next_item(a, iter);
        if (itx < 0) break;
        chunk_item<NJ, false, true>(a, itx, smem);
    }
}

// Two builds cover the three classes (class 8 runs in the nine-chunk build),
// and none stops frozen replicas: with UAVQ_STOP_FROZEN these classes sweep
// to the end, which gives the same outputs.
const void *chunk_sweep_big_kernel(int nj, bool stop) {
    (void)stop;
    if (nj == 7) return (const void *)k_sweep_chunk_big<7>;
    if (nj == 8 || nj == 9) return (const void *)k_sweep_chunk_big<9>;
    return nullptr;
}

}  // namespace uavq
