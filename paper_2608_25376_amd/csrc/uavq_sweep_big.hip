// Chunk classes 7..9 (m <= 576: fields up to 24x24), and every field whose
// travel costs exceed a byte (20x20 and larger at the default cost scale):
// the generic chunked walk with 16-bit costs read from global memory.  The
// cost matrix of a 24x24 field (575 cells) takes 661 KB, far beyond LDS, but
// fits an XCD's L2; LDS holds only the acceptance-table row.  The lane's
// step masks (up to 162 words) leave room for one wave per SIMD.
#include "uavq_factored.h"

namespace uavq {

template <int NJ, bool STOP>
__global__ __launch_bounds__(64 * kWideMaxWaves) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_sweep_factored_big(
    KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int iter = 0;; iter++) {
        const int itx = next_item(a, iter);
        if (itx < 0) break;
        factored_item<NJ, STOP, true>(a, itx, smem);
    }
}

// Two builds cover the three classes (class 8 runs in the nine-chunk build:
// more padding lanes, the same walk), and none stops frozen replicas: with
// UAVQ_STOP_FROZEN these classes sweep to the end, which gives the same
// outputs (each build takes minutes to compile).
const void *big_sweep_kernel(int nj, bool stop) {
    (void)stop;
    if (nj == 7) return (const void *)k_sweep_factored_big<7, false>;
    if (nj == 8 || nj == 9) return (const void *)k_sweep_factored_big<9, false>;
    return nullptr;
}

}  // namespace uavq
