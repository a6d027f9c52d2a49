// HIP kernels of libuavq for gfx950 (MI355X): replica initialisation, the
// factored and dense Metropolis sweeps, and the per-instance reduction.
//
// Model (paper Sec. III-B, eqs. (3)-(6), closed-tour reading): variables
// x_{t,c}, step t = 1..m, free cell c = 0..m-1.  The local field of site
// (t, c) has the structured form
//   h_{t,c} = -2P + 2P (R_t + C_c - 2 x_{t,c}) + Y_{t-1}[c] + Y_{t+1}[c]
// with R_t / C_c the step / cell occupation counts and Y_t = D^T x_t the
// travel-cost row of step t (Y_0 = Y_{m+1} = start-cell costs; Y_{m+1} = 0 for
// an open path).  A flip of (t, c*) changes, for the other sites of step t,
// only the 2P R_t term; it changes Y_t (used by steps t-1 and t+1) by the
// cost row of c*.
//
// Factored sweep, one replica per wavefront: the steps are visited in order;
// for step t every lane evaluates the sites of its own cells (c = lane + 64 j)
// against the current state, a ballot finds the first accepted site c* in
// site order, the flip is applied (O(m) update of Y_t) and evaluation resumes
// at c* + 1.  Sites before c* were rejections under an unchanged state and
// the random word of a site is addressed by (instance, replica, sweep, step,
// cell) rather than consumed, so the result equals the sequential sweep bit
// for bit.
//
// Replica state lives in registers: lane L holds the cell masks of steps
// L + 1 + 64 j (bits = cells) and the occupation count of cells L + 64 j.  The
// cost matrix D (bytes), the start-cell costs and a double-buffered row of the
// acceptance table live in LDS and are shared by the block's replicas.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "uavq_internal.h"

namespace uavq {

#define UAVQ_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return set_error(UAVQ_EHIP, "%s: %s", #call, hipGetErrorString(e_));         \
    } while (0)

static __host__ __device__ inline size_t al16(size_t v) { return (v + 15) & ~(size_t)15; }

// Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; i++) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint32_t pick4(uint4 v, int w) {
    return w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// ------------------------------------------------------------------ init --
// One block per work item; every unit (replica, 4-step block tb, word w)
// draws the 32 cells of that word for steps 4 tb + 1 .. 4 tb + 4 (stream 1).
__global__ __launch_bounds__(256) void k_init_states(KArgs a) {
    const WorkItem it = a.items[blockIdx.x];
    const InstDesc d = a.desc[it.inst];
    const int m = d.m, W = d.row_words, nb = (m + 3) >> 2;
    const int units = it.nrep * nb * W;
    for (int u = threadIdx.x; u < units; u += blockDim.x) {
        const int w = u % W;
        const int tb = (u / W) % nb;
        const int rl = u / (W * nb);
        const int r = it.rep0 + rl;
        const int64_t grep = d.rep_base + r;
        uint32_t *st = a.states + d.state_off + (int64_t)r * d.state_words;
        if (a.seeded && a.seeded[grep]) {
            // given state; bits of cells >= m are cleared
            const uint32_t *src = a.init_states + d.state_off + (int64_t)r * d.state_words;
            const int nbits = m - 32 * w;
            const uint32_t keep = nbits >= 32 ? 0xFFFFFFFFu : ((1u << nbits) - 1u);
            for (int k = 0; k < 4; k++) {
                const int t = 4 * tb + k + 1;
                if (t <= m) st[(t - 1) * W + w] = src[(t - 1) * W + w] & keep;
            }
            continue;
        }
        uint32_t rows[4] = {0u, 0u, 0u, 0u};
        for (int b = 0; b < 32; b++) {
            const int c = 32 * w + b;
            if (c >= m) break;
            const uint4 v = philox(make_uint4((uint32_t)c + 65536u * (uint32_t)tb, (uint32_t)r, d.inst_id, 0u),
                                   a.seed, 1u);
            rows[0] |= (v.x >> 31) << b;
            rows[1] |= (v.y >> 31) << b;
            rows[2] |= (v.z >> 31) << b;
            rows[3] |= (v.w >> 31) << b;
        }
        for (int k = 0; k < 4; k++) {
            const int t = 4 * tb + k + 1;
            if (t <= m) st[(t - 1) * W + w] = rows[k];
        }
    }
}

// --------------------------------------------------------- factored sweep --
template <int NJ>
struct RowOps {
    // mask of the step held by lane lt of one chunk of the step masks
    static __device__ __forceinline__ void read(const uint32_t (&rj)[2 * NJ], int lt, uint32_t (&out)[2 * NJ]) {
#pragma unroll
        for (int w = 0; w < 2 * NJ; w++) out[w] = __builtin_amdgcn_readlane(rj[w], lt);
    }
    static __device__ __forceinline__ void write(uint32_t (&rj)[2 * NJ], int lt, const uint32_t (&in)[2 * NJ], int L) {
        const bool mine = (L == lt);
#pragma unroll
        for (int w = 0; w < 2 * NJ; w++) rj[w] = mine ? in[w] : rj[w];
    }
    // Y[c] = sum over set cells c' of the mask of D[c'][c], for this lane's cells
    static __device__ __forceinline__ void costrow(const uint32_t (&mk)[2 * NJ], const uint8_t *sD, int m, int L,
                                                   int (&Y)[NJ]) {
#pragma unroll
        for (int j = 0; j < NJ; j++) Y[j] = 0;
#pragma unroll
        for (int w = 0; w < 2 * NJ; w++) {
            uint32_t bits = mk[w];
            while (bits) {
                const int b = __builtin_ctz(bits);
                bits &= bits - 1u;
                const uint8_t *row = sD + (32 * w + b) * m;
#pragma unroll
                for (int j = 0; j < NJ; j++) {
                    const int c = 64 * j + L;
                    if (c < m) Y[j] += row[c];
                }
            }
        }
    }
    static __device__ __forceinline__ int bit(const uint32_t (&mk)[2 * NJ], int j, int L) {
        const uint64_t v = ((uint64_t)mk[2 * j + 1] << 32) | (uint64_t)mk[2 * j];
        return (int)((v >> L) & 1ull);
    }
    static __device__ __forceinline__ int popc(const uint32_t (&mk)[2 * NJ]) {
        int r = 0;
#pragma unroll
        for (int w = 0; w < 2 * NJ; w++) r += __popc(mk[w]);
        return r;
    }
};

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NJ>
__global__ __launch_bounds__(1024) void k_sweep_factored(KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    using Ops = RowOps<NJ>;
    const WorkItem it = a.items[a.item_base + blockIdx.x];
    const InstDesc d = a.desc[it.inst];
    const int m = d.m, W = d.row_words, twoP = 2 * d.P;
    const int wave = threadIdx.x >> 6, L = threadIdx.x & 63;
    const int Dw = a.Dmax + 1;

    uint8_t *sD = smem;
    uint8_t *sdep = smem + al16((size_t)m * m);
    uint32_t *sthr = reinterpret_cast<uint32_t *>(smem + al16((size_t)m * m) + al16((size_t)m));
    __shared__ int s_first_sh;

    const uint8_t *gD = a.ws + d.d_off;
    const uint8_t *gdep = a.ws + d.ddep_off;
    for (int i = threadIdx.x; i < m * m; i += blockDim.x) sD[i] = gD[i];
    for (int i = threadIdx.x; i < m; i += blockDim.x) sdep[i] = gdep[i];

    const bool active = wave < it.nrep;
    const int r = it.rep0 + wave;
    const int64_t grep = d.rep_base + r;
    const int s0 = active ? (a.start_sweep ? a.start_sweep[grep] : 0) : a.S;
    if (threadIdx.x == 0) s_first_sh = a.S;
    __syncthreads();
    if (L == 0) atomicMin(&s_first_sh, s0);
    __syncthreads();
    const int s_first = s_first_sh;
    if (s_first < a.S) {
        const int n = a.dcut[s_first];
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            sthr[(s_first & 1) * Dw + i] = a.thr[(size_t)s_first * Dw + i];
    }
    __syncthreads();

    // ---- replica state into registers
    uint32_t rm[NJ][2 * NJ];
    int Cc[NJ];
    uint32_t *st = a.states + d.state_off + (int64_t)r * d.state_words;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int t = 64 * j + L + 1;
#pragma unroll
        for (int w = 0; w < 2 * NJ; w++) rm[j][w] = (active && t <= m && w < W) ? st[(t - 1) * W + w] : 0u;
        Cc[j] = 0;
    }
    // the best state starts as the initial state (kept if no sweep improves on +inf)
    if (active) {
        uint32_t *bs = a.best_states + d.state_off + (int64_t)r * d.state_words;
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            const int t = 64 * j + L + 1;
            if (t <= m)
#pragma unroll
                for (int w = 0; w < 2 * NJ; w++)
                    if (w < W) bs[(t - 1) * W + w] = rm[j][w];
        }
    }
    // occupation counts and initial energy (grouped pair sums of the QUBO)
    int64_t E = 0;
    if (active) {
        int64_t lane_e = 0, rowterm = 0;
        int Yp[NJ];
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            const int c = 64 * j + L;
            Yp[j] = c < m ? sdep[c] : 0;
        }
        uint32_t mk[2 * NJ];
#pragma unroll
        for (int jt = 0; jt < NJ; jt++)
        for (int lt = 0; lt < 64; lt++) {
            const int t = 64 * jt + lt + 1;
            if (t > m) break;
            Ops::read(rm[jt], lt, mk);
            const int R = Ops::popc(mk);
            rowterm += (int64_t)d.P * R * (R - 1) - (int64_t)twoP * R;
#pragma unroll
            for (int j = 0; j < NJ; j++) {
                const int x = Ops::bit(mk, j, L);
                Cc[j] += x;
                lane_e += x * Yp[j];
                if (t == m && d.closed && 64 * j + L < m) lane_e += x * (int)sdep[64 * j + L];
            }
            Ops::costrow(mk, sD, m, L, Yp);
        }
#pragma unroll
        for (int j = 0; j < NJ; j++) lane_e += (int64_t)d.P * Cc[j] * (Cc[j] - 1);
        E = d.c0 + rowterm + wave_sum64(lane_e);
    }

    int64_t bestE = LLONG_MAX;
    int bestS = -1;
    uint64_t nacc = 0, ndraw = 0;

    for (int s = s_first; s < a.S; s++) {
        const uint32_t *thr = sthr + (s & 1) * Dw;
        const int dcut = a.dcut[s];
        if (active && s >= s0) {
            int Yp[NJ], Yc[NJ], Yn[NJ];
#pragma unroll
            for (int j = 0; j < NJ; j++) {
                const int c = 64 * j + L;
                Yp[j] = c < m ? sdep[c] : 0;
            }
            uint32_t mc[2 * NJ], mn[2 * NJ];
            Ops::read(rm[0], 0, mc);
            Ops::costrow(mc, sD, m, L, Yc);
            int blk = -1;
            uint4 u4[NJ];
#pragma unroll
            for (int jt = 0; jt < NJ; jt++)
            for (int lt = 0; lt < 64; lt++) {
                const int t = 64 * jt + lt + 1;
                if (t > m) break;
                if (t < m) {
                    if (lt < 63) Ops::read(rm[jt], lt + 1, mn);
                    else Ops::read(rm[jt + 1 < NJ ? jt + 1 : jt], 0, mn);
                    Ops::costrow(mn, sD, m, L, Yn);
                } else {
#pragma unroll
                    for (int j = 0; j < NJ; j++) {
                        const int c = 64 * j + L;
                        Yn[j] = (d.closed && c < m) ? sdep[c] : 0;
                    }
                }
                int R = Ops::popc(mc);
                int x[NJ], base[NJ];
#pragma unroll
                for (int j = 0; j < NJ; j++) {
                    x[j] = Ops::bit(mc, j, L);
                    base[j] = Yp[j] + Yn[j] + twoP * (Cc[j] - 2 * x[j]) - twoP;
                }
                int start = 0;
                bool changed = false;
                while (true) {
                    const int hR = twoP * R;
                    bool acc[NJ], need[NJ];
                    int dE[NJ];
                    uint64_t needm[NJ];
                    bool any_need = false;
#pragma unroll
                    for (int j = 0; j < NJ; j++) {
                        const int c = 64 * j + L;
                        const int h = base[j] + hR;
                        dE[j] = x[j] ? -h : h;
                        const bool valid = (c >= start) && (c < m);
                        acc[j] = valid && dE[j] <= 0;
                        need[j] = valid && dE[j] > 0 && dE[j] < dcut;
                        needm[j] = ballot64(need[j]);
                        any_need |= needm[j] != 0;
                    }
                    if (any_need) {
                        const int tb = (t - 1) >> 2;
                        if (blk != tb) {
#pragma unroll
                            for (int j = 0; j < NJ; j++)
                                u4[j] = philox(make_uint4((uint32_t)(64 * j + L) + 65536u * (uint32_t)tb, (uint32_t)s,
                                                          (uint32_t)r, d.inst_id),
                                               a.seed, 0u);
                            blk = tb;
                        }
                        const int wsel = (t - 1) & 3;
#pragma unroll
                        for (int j = 0; j < NJ; j++)
                            if (need[j]) acc[j] = pick4(u4[j], wsel) < thr[dE[j]];
                    }
                    int cstar = -1;
#pragma unroll
                    for (int j = 0; j < NJ; j++) {
                        const uint64_t am = ballot64(acc[j]);
                        if (cstar < 0 && am) cstar = 64 * j + __builtin_ctzll(am);
                    }
                    if (cstar < 0) {
#pragma unroll
                        for (int j = 0; j < NJ; j++) ndraw += __popcll(needm[j]);
                        break;
                    }
                    // draws taken at sites start .. cstar
                    const int jstar = cstar >> 6, Lstar = cstar & 63;
#pragma unroll
                    for (int j = 0; j < NJ; j++) {
                        if (j < jstar) ndraw += __popcll(needm[j]);
                        else if (j == jstar)
                            ndraw += __popcll(needm[j] & (Lstar == 63 ? ~0ull : ((2ull << Lstar) - 1ull)));
                    }
                    // apply the flip of (t, cstar)
                    const int wstar = cstar >> 5;
                    const uint32_t bstar_bit = 1u << (cstar & 31);
                    int xs = 0;
#pragma unroll
                    for (int w = 0; w < 2 * NJ; w++)
                        if (w == wstar) xs = (mc[w] & bstar_bit) ? 1 : 0;
                    const int sign = xs ? -1 : 1;
                    int bstar = 0;
#pragma unroll
                    for (int j = 0; j < NJ; j++)
                        if (j == jstar) bstar = __builtin_amdgcn_readlane(base[j], Lstar);
                    const int hstar = bstar + hR;
                    E += (int64_t)(xs ? -hstar : hstar);
                    nacc++;
#pragma unroll
                    for (int w = 0; w < 2 * NJ; w++)
                        if (w == wstar) mc[w] ^= bstar_bit;
                    R += sign;
                    changed = true;
                    const uint8_t *drow = sD + cstar * m;
#pragma unroll
                    for (int j = 0; j < NJ; j++) {
                        const int c = 64 * j + L;
                        if (j == jstar && L == Lstar) {
                            Cc[j] += sign;
                            x[j] ^= 1;
                        }
                        if (c < m) Yc[j] += sign * (int)drow[c];
                    }
                    start = cstar + 1;
                    if (start >= m) break;
                }
                if (changed) Ops::write(rm[jt], lt, mc, L);
#pragma unroll
                for (int j = 0; j < NJ; j++) {
                    Yp[j] = Yc[j];
                    Yc[j] = Yn[j];
                }
#pragma unroll
                for (int w = 0; w < 2 * NJ; w++) mc[w] = mn[w];
            }
            if (E < bestE) {
                bestE = E;
                bestS = s;
                uint32_t *bs = a.best_states + d.state_off + (int64_t)r * d.state_words;
#pragma unroll
                for (int j = 0; j < NJ; j++) {
                    const int t = 64 * j + L + 1;
                    if (t <= m)
#pragma unroll
                        for (int w = 0; w < 2 * NJ; w++)
                            if (w < W) bs[(t - 1) * W + w] = rm[j][w];
                }
            }
        }
        if (s + 1 < a.S) {
            const int n = a.dcut[s + 1];
            uint32_t *dst = sthr + ((s + 1) & 1) * Dw;
            const uint32_t *src = a.thr + (size_t)(s + 1) * Dw;
            for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
        }
        __syncthreads();
    }

    if (active) {
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            const int t = 64 * j + L + 1;
            if (t <= m)
#pragma unroll
                for (int w = 0; w < 2 * NJ; w++)
                    if (w < W) st[(t - 1) * W + w] = rm[j][w];
        }
        if (L == 0) {
            a.final_E[grep] = E;
            a.best_E[grep] = bestE;
            a.best_sweep[grep] = bestS;
            a.accepts[grep] = nacc;
            a.draws[grep] = ndraw;
        }
    }
}

// ------------------------------------------------------------ reduction --
// Per instance: lexicographic minimum of (best_E, replica), then copy of the
// winner's best state.
__global__ __launch_bounds__(256) void k_reduce(KArgs a) {
    const int inst = blockIdx.x;
    const InstDesc d = a.desc[inst];
    __shared__ int64_t sE[256];
    __shared__ int sR[256];
    int64_t bE = LLONG_MAX;
    int bR = INT_MAX;
    for (int r = threadIdx.x; r < d.nrep; r += blockDim.x) {
        const int64_t e = a.best_E[d.rep_base + r];
        if (e < bE || (e == bE && r < bR)) {
            bE = e;
            bR = r;
        }
    }
    sE[threadIdx.x] = bE;
    sR[threadIdx.x] = bR;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            const int64_t e2 = sE[threadIdx.x + off];
            const int r2 = sR[threadIdx.x + off];
            if (e2 < sE[threadIdx.x] || (e2 == sE[threadIdx.x] && r2 < sR[threadIdx.x])) {
                sE[threadIdx.x] = e2;
                sR[threadIdx.x] = r2;
            }
        }
        __syncthreads();
    }
    const int win = sR[0];
    if (threadIdx.x == 0) {
        if (a.inst_best_E) a.inst_best_E[inst] = sE[0];
        if (a.inst_best_replica) a.inst_best_replica[inst] = win;
        if (a.inst_best_sweep) a.inst_best_sweep[inst] = a.best_sweep[d.rep_base + win];
    }
    if (a.inst_best_state) {
        const uint32_t *src = a.best_states + d.state_off + (int64_t)win * d.state_words;
        uint32_t *dst = a.inst_best_state + a.inst_state_off[inst];
        for (int i = threadIdx.x; i < d.state_words; i += blockDim.x) dst[i] = src[i];
    }
}

// ------------------------------------------------------------- launchers --
template <int NJ>
static int launch_factored_class(const uavq_plan *pl, KArgs a, int cls, hipStream_t st) {
    const int b0 = pl->class_begin[cls], b1 = pl->class_begin[cls + 1];
    if (b1 <= b0) return UAVQ_OK;
    int mmax = 0;
    for (int i = b0; i < b1; i++) mmax = std::max(mmax, pl->desc[pl->items[i].inst].m);
    const size_t lds = al16((size_t)mmax * mmax) + al16((size_t)mmax) + 2 * (size_t)(pl->Dmax + 1) * 4;
    if (lds > 160 * 1024)
        return set_error(UAVQ_ETOOBIG, "anneal: LDS need %zu bytes (m = %d, Dmax = %d)", lds, mmax, pl->Dmax);
    UAVQ_HIP(hipFuncSetAttribute((const void *)k_sweep_factored<NJ>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
    a.item_base = b0;
    const int wpb = pl->waves_per_block[cls];
    if (pl->timing) UAVQ_HIP(hipEventRecord((hipEvent_t)pl->ev[2 * cls], st));
    hipLaunchKernelGGL(k_sweep_factored<NJ>, dim3(b1 - b0), dim3(64 * wpb), lds, st, a);
    if (pl->timing) UAVQ_HIP(hipEventRecord((hipEvent_t)pl->ev[2 * cls + 1], st));
    UAVQ_HIP(hipGetLastError());
    return UAVQ_OK;
}

int launch_anneal(const uavq_plan *pl, const KArgs &a0, void *stream, int64_t *check_E) {
    hipStream_t st = (hipStream_t)stream;
    KArgs a = a0;
    const int n_items = (int)pl->items.size();
    if (n_items == 0) return UAVQ_OK;
    if (check_E) return set_error(UAVQ_EINVAL, "anneal: check_E not supported yet");
    if (pl->dense) return set_error(UAVQ_EINVAL, "anneal: dense kernel not built yet");
    a.item_base = 0;
    hipLaunchKernelGGL(k_init_states, dim3(n_items), dim3(256), 0, st, a);
    UAVQ_HIP(hipGetLastError());
    int rc;
    if ((rc = launch_factored_class<1>(pl, a, 1, st))) return rc;
    if ((rc = launch_factored_class<2>(pl, a, 2, st))) return rc;
    if ((rc = launch_factored_class<3>(pl, a, 3, st))) return rc;
    hipLaunchKernelGGL(k_reduce, dim3(pl->n_inst), dim3(256), 0, st, a);
    UAVQ_HIP(hipGetLastError());
    return UAVQ_OK;
}

size_t energy_ws_bytes(const uavq_qubo *q) { return q ? 256 : 0; }

int launch_energy(const uavq_qubo *, const uint32_t *, int64_t, int64_t *, void *, size_t, void *) {
    return set_error(UAVQ_EINVAL, "energy_eval_dev: not built yet");
}

}  // namespace uavq

using namespace uavq;

extern "C" {

int uavq_plan_upload(const uavq_plan *pl, void *d_ws, size_t ws_bytes, void *stream) {
    if (!pl || !d_ws) return set_error(UAVQ_EINVAL, "plan_upload: null argument");
    if (ws_bytes < pl->ws_bytes) return set_error(UAVQ_EINVAL, "plan_upload: workspace %zu < %zu bytes", ws_bytes, pl->ws_bytes);
    UAVQ_HIP(hipMemcpyAsync(d_ws, pl->blob.data(), pl->blob.size(), hipMemcpyHostToDevice, (hipStream_t)stream));
    return UAVQ_OK;
}

int uavq_anneal_batch(const uavq_plan *pl, void *d_ws, size_t ws_bytes, const uavq_anneal_init *init,
                      const uavq_anneal_out *out, void *stream) {
    if (!pl || !out) return set_error(UAVQ_EINVAL, "anneal_batch: null argument");
    if (pl->total_rep == 0) return UAVQ_OK;
    if (!d_ws || ws_bytes < pl->ws_bytes) return set_error(UAVQ_EINVAL, "anneal_batch: workspace too small");
    if (!out->final_states || !out->final_E || !out->best_E || !out->best_sweep || !out->best_states ||
        !out->accepts || !out->draws)
        return set_error(UAVQ_EINVAL, "anneal_batch: a required output is NULL");
    if (init && init->seeded && !init->states)
        return set_error(UAVQ_EINVAL, "anneal_batch: seeded replicas need init->states");
    KArgs a{};
    const uint8_t *ws = (const uint8_t *)d_ws;
    a.ws = ws;
    a.desc = (const InstDesc *)(ws + pl->desc_off);
    a.items = (const WorkItem *)(ws + pl->items_off);
    a.n_items = (int32_t)pl->items.size();
    a.thr = (const uint32_t *)(ws + pl->thr_off);
    a.dcut = (const int32_t *)(ws + pl->dcut_off);
    a.S = pl->S;
    a.Dmax = pl->Dmax;
    a.seed = pl->p.seed;
    a.n_inst = pl->n_inst;
    a.total_rep = pl->total_rep;
    if (init) {
        a.init_states = init->states;
        a.seeded = init->seeded;
        a.start_sweep = init->start_sweep;
    }
    a.states = out->final_states;
    a.E_init = (int64_t *)(ws + pl->e_init_off);
    a.final_E = out->final_E;
    a.best_E = out->best_E;
    a.best_sweep = out->best_sweep;
    a.best_states = out->best_states;
    a.accepts = out->accepts;
    a.draws = out->draws;
    a.inst_best_E = out->inst_best_E;
    a.inst_best_replica = out->inst_best_replica;
    a.inst_best_sweep = out->inst_best_sweep;
    a.inst_best_state = out->inst_best_state;
    a.inst_state_off = (int64_t *)(ws + pl->inst_state_off_off);
    return launch_anneal(pl, a, stream, out->check_E);
}

int uavq_plan_set_timing(uavq_plan *pl, int32_t enable) {
    if (!pl) return set_error(UAVQ_EINVAL, "plan_set_timing: null plan");
    if (enable && !pl->ev[0]) {
        for (int i = 0; i < 2 * (kMaxChunks + 1); i++) {
            hipEvent_t e;
            UAVQ_HIP(hipEventCreate(&e));
            pl->ev[i] = (void *)e;
        }
    }
    pl->timing = enable ? 1 : 0;
    return UAVQ_OK;
}

int uavq_plan_sweep_ms(const uavq_plan *pl, float *ms) {
    if (!pl || !ms) return set_error(UAVQ_EINVAL, "plan_sweep_ms: null argument");
    if (!pl->timing) return set_error(UAVQ_EINVAL, "plan_sweep_ms: timing not enabled");
    float total = 0.f;
    for (int cls = 1; cls <= kMaxChunks; cls++) {
        if (pl->class_begin[cls + 1] <= pl->class_begin[cls]) continue;
        float t = 0.f;
        UAVQ_HIP(hipEventElapsedTime(&t, (hipEvent_t)pl->ev[2 * cls], (hipEvent_t)pl->ev[2 * cls + 1]));
        total += t;
    }
    *ms = total;
    return UAVQ_OK;
}

void plan_destroy_events(uavq_plan *pl) {
    for (int i = 0; i < 2 * (kMaxChunks + 1); i++)
        if (pl->ev[i]) {
            (void)hipEventDestroy((hipEvent_t)pl->ev[i]);
            pl->ev[i] = nullptr;
        }
}

int uavq_energy_workspace_bytes(const uavq_qubo *q, size_t *bytes) {
    if (!q || !bytes) return set_error(UAVQ_EINVAL, "energy_workspace_bytes: null argument");
    *bytes = energy_ws_bytes(q);
    return UAVQ_OK;
}

int uavq_energy_eval_dev(const uavq_qubo *q, const uint32_t *d_x, int64_t n, int64_t *d_E, void *d_ws,
                         size_t ws_bytes, void *stream) {
    if (!q || n < 0 || (n > 0 && (!d_x || !d_E))) return set_error(UAVQ_EINVAL, "energy_eval_dev: bad argument");
    if (n == 0) return UAVQ_OK;
    return launch_energy(q, d_x, n, d_E, d_ws, ws_bytes, stream);
}

}  // extern "C"
