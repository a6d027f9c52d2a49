// Replica exchange between neighbouring slots of a parallel-tempering ladder.
//
// Chain r has K slots at fixed temperatures T_0 > ... > T_{K-1}; slot k's
// states and energies are the final_states / final_E of its own plan, laid
// out slot-major ([K][R][words], [K][R]).  A round visits the pairs
// (k, k+1), k = round mod 2, k + 2, ...: with d = E_{k+1} - E_k the swap is
// taken when d >= 0, else when u < xthr[k][min(-d, DX[k])] (a zero entry needs
// no draw), u = word 0 of Philox({k, round, r, inst}, {seed, 5}).  The table
// holds floor(2^32 exp(-a (1/T_{k+1} - 1/T_k))), so the swap probability is
// min(1, exp((1/T_{k+1} - 1/T_k) d)): the Metropolis rule on the product of
// the two Boltzmann weights.  Integer decisions only.
//
// One wave per (pair, chain): every lane evaluates the same decision from the
// same two energies, then the lanes swap the two state rows word by word
// (coalesced; 4 waves per workgroup).  The round touches 2 energies and one
// table entry per pair, and the state rows only of accepted swaps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "uavq_device.h"
#include "uavq_internal.h"

namespace uavq {

struct PtArgs {
    const int32_t *DX;
    const uint32_t *xthr;
    int32_t *states;
    int64_t *E;
    unsigned long long *swaps;
    int32_t K, R, W, stride;
    uint32_t round, seed, inst;
};

__global__ __launch_bounds__(256) void k_pt_exchange(PtArgs a) {
    const int lane = threadIdx.x & 63;
    const int r = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int k = (int)(a.round & 1u) + 2 * (int)blockIdx.y;
    if (r >= a.R || k + 1 >= a.K) return;
    int64_t *Eh = a.E + (int64_t)k * a.R + r;
    int64_t *Ec = Eh + a.R;
    const int64_t eh = *Eh, ec = *Ec;
    const int64_t d = ec - eh;
    bool swap = d >= 0;
    if (!swap) {
        const int64_t dx = (int64_t)min(a.DX[k], a.stride - 1);
        const int64_t am = -d < dx ? -d : dx;
        const uint32_t th = a.xthr[(int64_t)k * a.stride + am];
        swap = th != 0u && philox(make_uint4((uint32_t)k, a.round, (uint32_t)r, a.inst), a.seed, 5u).x < th;
    }
    if (!swap) return;
    int32_t *xh = a.states + ((int64_t)k * a.R + r) * a.W;
    int32_t *xc = xh + (int64_t)a.R * a.W;
    for (int w = lane; w < a.W; w += 64) {
        const int32_t t = xh[w];
        xh[w] = xc[w];
        xc[w] = t;
    }
    if (lane == 0) {
        *Eh = ec;
        *Ec = eh;
        if (a.swaps) atomicAdd(a.swaps + k, 1ull);
    }
}

// The same round over a batch of chain sets (blockIdx.z = set), each with its
// own state offset, state width and instance id.
struct PtBatchArgs {
    const int64_t *state_off;
    const int32_t *words;
    const uint32_t *inst;
    const int32_t *DX;
    const uint32_t *xthr;
    int32_t *states;
    int64_t *E;
    unsigned long long *swaps;
    int32_t K, R, stride;
    uint32_t round, seed;
};

__global__ __launch_bounds__(256) void k_pt_exchange_batch(PtBatchArgs a) {
    const int lane = threadIdx.x & 63;
    const int r = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int k = (int)(a.round & 1u) + 2 * (int)blockIdx.y;
    const int set = (int)blockIdx.z;
    if (r >= a.R || k + 1 >= a.K) return;
    const int W = a.words[set];
    int64_t *Eh = a.E + ((int64_t)set * a.K + k) * a.R + r;
    int64_t *Ec = Eh + a.R;
    const int64_t eh = *Eh, ec = *Ec;
    const int64_t d = ec - eh;
    bool swap = d >= 0;
    if (!swap) {
        const int64_t dx = (int64_t)min(a.DX[k], a.stride - 1);
        const int64_t am = -d < dx ? -d : dx;
        const uint32_t th = a.xthr[(int64_t)k * a.stride + am];
        swap = th != 0u && philox(make_uint4((uint32_t)k, a.round, (uint32_t)r, a.inst[set]), a.seed, 5u).x < th;
    }
    if (!swap) return;
    int32_t *xh = a.states + a.state_off[set] + ((int64_t)k * a.R + r) * W;
    int32_t *xc = xh + (int64_t)a.R * W;
    for (int w = lane; w < W; w += 64) {
        const int32_t t = xh[w];
        xh[w] = xc[w];
        xc[w] = t;
    }
    if (lane == 0) {
        *Eh = ec;
        *Ec = eh;
        if (a.swaps) atomicAdd(a.swaps + (int64_t)set * (a.K - 1) + k, 1ull);
    }
}

}  // namespace uavq

using namespace uavq;

extern "C" int uavq_pt_exchange_batch(int32_t n_sets, int32_t K, int32_t R, uint32_t round, uint32_t seed,
                                      const int64_t *d_state_off, const int32_t *d_words, const uint32_t *d_inst,
                                      const int32_t *d_DX, const uint32_t *d_xthr, int32_t stride, int32_t *d_states,
                                      int64_t *d_E, uint64_t *d_swaps, void *stream) {
    if (n_sets < 1 || n_sets > 65535) return set_error(UAVQ_EINVAL, "pt_exchange_batch: n_sets = %d outside 1..65535", n_sets);
    if (K < 1 || K > 4096) return set_error(UAVQ_EINVAL, "pt_exchange_batch: K = %d outside 1..4096", K);
    if (R < 1 || R > (1 << 20)) return set_error(UAVQ_EINVAL, "pt_exchange_batch: R = %d outside 1..2^20", R);
    if (stride < 2) return set_error(UAVQ_EINVAL, "pt_exchange_batch: stride >= 2");
    if (!d_state_off || !d_words || !d_inst || !d_DX || !d_xthr || !d_states || !d_E)
        return set_error(UAVQ_EINVAL, "pt_exchange_batch: null pointer");
    const int32_t pairs = (K - (int32_t)(round & 1u)) / 2;
    if (pairs < 1) return UAVQ_OK;
    PtBatchArgs a{d_state_off, d_words, d_inst, d_DX, d_xthr, d_states, d_E, (unsigned long long *)d_swaps,
                  K, R, stride, round, seed};
    hipLaunchKernelGGL(k_pt_exchange_batch, dim3((unsigned)((R + 3) / 4), (unsigned)pairs, (unsigned)n_sets), dim3(256),
                       0, (hipStream_t)stream, a);
    UAVQ_HIP(hipGetLastError());
    return UAVQ_OK;
}

extern "C" int uavq_pt_exchange(int32_t K, int32_t R, int32_t state_words, uint32_t round, uint32_t seed,
                                uint32_t inst_id, const int32_t *d_DX, const uint32_t *d_xthr, int32_t stride,
                                int32_t *d_states, int64_t *d_E, uint64_t *d_swaps, void *stream) {
    if (K < 1 || K > 4096) return set_error(UAVQ_EINVAL, "pt_exchange: K = %d outside 1..4096", K);
    if (R < 1 || R > (1 << 20)) return set_error(UAVQ_EINVAL, "pt_exchange: R = %d outside 1..2^20", R);
    if (state_words < 1 || stride < 2) return set_error(UAVQ_EINVAL, "pt_exchange: state_words >= 1, stride >= 2");
    if (!d_DX || !d_xthr || !d_states || !d_E) return set_error(UAVQ_EINVAL, "pt_exchange: null pointer");
    const int32_t pairs = (K - (int32_t)(round & 1u)) / 2;
    if (pairs < 1) return UAVQ_OK;
    PtArgs a{d_DX, d_xthr, d_states, d_E, (unsigned long long *)d_swaps, K, R, state_words, stride, round, seed,
             inst_id};
    hipLaunchKernelGGL(k_pt_exchange, dim3((unsigned)((R + 3) / 4), (unsigned)pairs), dim3(256), 0,
                       (hipStream_t)stream, a);
    UAVQ_HIP(hipGetLastError());
    return UAVQ_OK;
}
