// The generic chunked factored sweep (any m <= 64 * kMaxChunks), shared by
// the translation units that instantiate it: lane L holds the cell masks of
// steps L + 1 + 64 j and the occupation counts of cells L + 64 j; travel rows
// are rebuilt from the neighbouring steps' masks.  DG = true reads the cost
// matrix as 16-bit entries from global memory (L2) instead of bytes in LDS,
// for fields whose costs exceed a byte or whose matrix leaves no room in LDS.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>

#include "uavq_device.h"

namespace uavq {

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
    template <typename DT>
    static __device__ __forceinline__ void costrow(const uint32_t (&mk)[2 * NJ], const DT *sD, int m, int L,
                                                   int (&Y)[NJ]) {
#pragma unroll
        for (int j = 0; j < NJ; j++) Y[j] = 0;
#pragma unroll
        for (int w = 0; w < 2 * NJ; w++) {
            uint32_t bits = mk[w];
            while (bits) {
                const int b = __builtin_ctz(bits);
                bits &= bits - 1u;
                const DT *row = sD + (32 * w + b) * m;
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


// uint4 chunks of the next acceptance-table row held in registers while a
// sweep runs (the rest, for small blocks, is copied directly).
template <int NJ>
struct Prefetch {
    static constexpr int K = NJ == 1 ? 6 : (NJ == 2 ? 4 : 2);
};

// STOP: built with UAVQ_STOP_FROZEN (a replica whose sweep had neither an
// accept nor a draw sweeps no more; the block leaves when all have stopped).
// DG: the cost matrix and start-cell costs are 16-bit entries in global memory
// (read through L2; lanes past m read up to 64 kMaxChunks entries beyond the
// matrix, which the plan pads), and LDS holds only the table row.
template <int NJ, bool STOP, bool DG = false>
__device__ __forceinline__ void factored_item(const KArgs &a, int itx, uint8_t *smem) {
    using DT = typename std::conditional<DG, uint16_t, uint8_t>::type;
    using Ops = RowOps<NJ>;
    constexpr int KP = Prefetch<NJ>::K;
    const WorkItem it = a.items[itx];
    const InstDesc d = a.desc[it.inst];
    const int m = d.m, W = d.row_words, twoP = 2 * d.P;
    const int wave = threadIdx.x >> 6, L = threadIdx.x & 63;
    const int nthr = blockDim.x;
    const int Ts = a.thr_stride;   // row stride of the acceptance table, a multiple of 4
    // this instance's schedule: sweep s reads table row sched_row + s * sched_step
    const int srow = d.sched_row, dstep = d.sched_step;

    // LDS: the acceptance-table row | D (m*m bytes) | start-cell costs (m bytes)
    uint32_t *sthr = reinterpret_cast<uint32_t *>(smem);
    const DT *sD = DG ? reinterpret_cast<const DT *>(a.ws + d.d_off) : reinterpret_cast<const DT *>(smem + 4 * (size_t)Ts);
    const DT *sdep = DG ? reinterpret_cast<const DT *>(a.ws + d.ddep_off) : sD + al16((size_t)m * m);
    __shared__ int s_first_sh;
    __shared__ int s_live[2];   // replicas of the block that can still change, by sweep parity

    {
        const uint4 *gD = reinterpret_cast<const uint4 *>(a.ws + d.d_off);
        const uint4 *gdep = reinterpret_cast<const uint4 *>(a.ws + d.ddep_off);
        const int nD4 = (m * m + 15) >> 4, nd4 = (m + 15) >> 4;
        uint8_t *lD = smem + 4 * (size_t)Ts, *ldep = lD + al16((size_t)m * m);
        if (!DG) {
            for (int i = threadIdx.x; i < nD4; i += nthr) reinterpret_cast<uint4 *>(lD)[i] = gD[i];
            for (int i = threadIdx.x; i < nd4; i += nthr) reinterpret_cast<uint4 *>(ldep)[i] = gdep[i];
        }
    }

    const bool active = wave < it.nrep;
    const int r = it.rep0 + wave;
    const int64_t grep = d.rep_base + r;
    const int s0 = active ? max(a.start_sweep ? a.start_sweep[grep] : 0, a.s_begin) : a.s_end;
    if (threadIdx.x == 0) {
        s_first_sh = a.s_end;
        if (STOP) s_live[0] = s_live[1] = 0;
    }
    __syncthreads();
    if (L == 0) atomicMin(&s_first_sh, s0);
    __syncthreads();
    const int s_first = s_first_sh;
    if (s_first < a.s_end) {
        const int n4 = (a.dcut[srow + s_first * dstep] + 2 + 3) >> 2;   // through index dcut + 1
        const uint4 *src = reinterpret_cast<const uint4 *>(a.thr + (size_t)(srow + s_first * dstep) * Ts);
        uint4 *dst = reinterpret_cast<uint4 *>(sthr);
        for (int i = threadIdx.x; i < n4; i += nthr) dst[i] = src[i];
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
    if (active && !a.resume) {
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

    // best so far and counters: fresh, or those of the previous segment
    int64_t bestE = LLONG_MAX;
    int bestS = -1;
    uint64_t nacc = 0, ndraw = 0;   // this launch's counts (a resumed run adds the stored ones at the end)
    if (active && a.resume) {
        bestE = a.best_E[grep];
        bestS = a.best_sweep[grep];
    }
    int64_t Elane = 0;         // energy change of the lane's accepted flips in the current sweep
    uint32_t ndraw_lane = 0;   // draws of the lane's sites
    bool frozen = false;       // stop_frozen: a sweep had neither an accept nor a draw
    int dep[NJ];   // start-cell costs of this lane's cells (the fixed rows 0 and m+1)
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int c = 64 * j + L;
        dep[j] = c < m ? sdep[c] : 0;
    }

    for (int s = s_first; s < a.s_end; s++) {
        // next table row: loads issued now, stored to LDS after this sweep
        uint4 pre[KP];
        const bool has_next = s + 1 < a.s_end;
        const int n4_next = has_next ? (uniform_load(a.dcut, srow + (s + 1) * dstep) + 2 + 3) >> 2 : 0;
        const uint4 *src_next = reinterpret_cast<const uint4 *>(a.thr + (size_t)(srow + (s + 1) * dstep) * Ts);
#pragma unroll
        for (int k = 0; k < KP; k++) {
            const int i = threadIdx.x + k * nthr;
            pre[k] = has_next ? src_next[i < n4_next ? i : 0] : make_uint4(0u, 0u, 0u, 0u);
        }
        const uint32_t *thr = sthr;
        const int dcut = uniform_load(a.dcut, srow + s * dstep);
        const float tl2 = __builtin_amdgcn_exp2f(d.tl2_a + d.tl2_b * (float)s);   // ~ T_s ln 2
        const float e0 = 32.0f * tl2 - 0.5f, dm1 = (float)(dcut - 1);
        if (STOP && threadIdx.x == 0) s_live[(s + 1) & 1] = 0;   // its last reader passed the previous sweep's barriers
        if (active && s >= s0 && !frozen) {
            const uint32_t ndl0 = STOP ? ndraw_lane : 0u;
            // Yp = Y_{t-1} (final), Yc = Y_t (updated on flips), Yn = Y_{t+1}, Ynn = Y_{t+2}
            int Yp[NJ], Yc[NJ], Yn[NJ], Ynn[NJ];
            uint32_t mc[2 * NJ], mn[2 * NJ], mnn[2 * NJ];
#pragma unroll
            for (int j = 0; j < NJ; j++) Yp[j] = dep[j];
            Ops::read(rm[0], 0, mc);
            Ops::costrow(mc, sD, m, L, Yc);
            if (m >= 2) {
                Ops::read(rm[0], 1, mn);
                Ops::costrow(mn, sD, m, L, Yn);
            } else {
#pragma unroll
                for (int w = 0; w < 2 * NJ; w++) mn[w] = 0u;
#pragma unroll
                for (int j = 0; j < NJ; j++) Yn[j] = d.closed ? dep[j] : 0;
            }
            int blk = -1;
            uint32_t have_cut = 0;   // bit j: chunk j's cuts of the current block are known
            uint32_t cutp[NJ][2];    // the block's cuts per chunk, two 16-bit values per word (cut <= dcut < 2^16)
            uint32_t nacc_s = 0;
#pragma unroll
            for (int jt = 0; jt < NJ; jt++)
                for (int lt = 0; lt < 64; lt++) {
                    const int t = 64 * jt + lt + 1;
                    if (t > m) break;
                    // look-ahead: Y_{t+2} from step t+2, unchanged until that step is visited
                    if (t + 2 <= m) {
                        const int q2 = lt + 2;
                        if (q2 < 64) Ops::read(rm[jt], q2, mnn);
                        else Ops::read(rm[jt + 1 < NJ ? jt + 1 : jt], q2 - 64, mnn);
                        Ops::costrow(mnn, sD, m, L, Ynn);
                    } else {
#pragma unroll
                        for (int w = 0; w < 2 * NJ; w++) mnn[w] = 0u;
#pragma unroll
                        for (int j = 0; j < NJ; j++) Ynn[j] = d.closed ? dep[j] : 0;
                    }
                    // ---- step t.  x, R_t and dE0 (dE against the state at the step
                    // start) per lane and chunk; the walk then moves a uniform count
                    // k of net 1s gained by the step, so every open site's dE is
                    // dE0 + k dplus (cf. the m <= 64 sweep)
                    const int hR0 = twoP * Ops::popc(mc);
                    int dE0[NJ];
#pragma unroll
                    for (int j = 0; j < NJ; j++) {
                        const int xj = Ops::bit(mc, j, L);
                        const int h = Yp[j] + Yn[j] + twoP * (Cc[j] - 2 * xj) - twoP + hR0;
                        dE0[j] = xj ? -h : h;
                    }
                    // change of dE per net 1 gained by step t (x read from the step mask)
                    auto dplus = [&](int j) { return Ops::bit(mc, j, L) ? -twoP : twoP; };
                    const int tb = (t - 1) >> 2, ti = (t - 1) & 3;
                    if (blk != tb) {   // a new block of four steps: its words and cuts are not drawn yet
                        blk = tb;
                        have_cut = 0;
                    }
                    int k = 0, psg = 0;
                    uint64_t accd[NJ];
                    int dY[NJ], pd[NJ];   // travel-row change; cost-row entries of the last flip
#pragma unroll
                    for (int j = 0; j < NJ; j++) {
                        accd[j] = 0;
                        dY[j] = 0;
                        pd[j] = 0;
                    }
                    // flip the first accepted site of chunk j's mask am; its cost-row
                    // entries are read now and added at the next flip
                    auto flip = [&](int j, uint64_t am, uint64_t &openm) {
                        const int Ls = __builtin_ctzll(am);
                        accd[j] |= 1ull << Ls;
                        const uint64_t rowj = ((uint64_t)mc[2 * j + 1] << 32) | (uint64_t)mc[2 * j];
                        const bool clears = (rowj >> Ls) & 1ull;
#pragma unroll
                        for (int jj = 0; jj < NJ; jj++) dY[jj] += __mul24(psg, pd[jj]);
                        // lanes past m read bytes beyond the row (inside the allocation); unused
                        const DT *drow = sD + (64 * j + Ls) * m;
#pragma unroll
                        for (int jj = 0; jj < NJ; jj++) pd[jj] = drow[64 * jj + L];
                        psg = clears ? -1 : 1;
                        k += psg;
                        openm &= ~1ull << Ls;
                    };
                    // a step with no valid site below the cut is finished: no accept, no draw
                    int mnv = INT_MAX;
#pragma unroll
                    for (int j = 0; j < NJ; j++) mnv = min(mnv, 64 * j + L < m ? dE0[j] : INT_MAX);
                    const bool cold = !ballot64(mnv < dcut);
#pragma unroll
                    for (int j = 0; j < NJ; j++) {
                        if (cold || 64 * j >= m) break;
                        uint64_t openm = m - 64 * j >= 64 ? ~0ull : ((1ull << (m - 64 * j)) - 1ull);
                        bool walking = true;
                        if (!((have_cut >> j) & 1u)) {
                            // no exact cut yet: accept iff dE <= 0 while no open site of the
                            // chunk needs a draw; then the chunk's words and cuts are drawn
                            while (true) {
                                const int dE = dE0[j] + __mul24(k, dplus(j));
                                if (ballot64((uint32_t)(dE - 1) < (uint32_t)(dcut - 1)) & openm) {
                                    have_cut |= 1u << j;
                                    uint32_t cbase = (uint32_t)(64 * j + L) + 65536u * (uint32_t)tb;
                                    asm volatile("" : "+v"(cbase));   // generator stays inside this branch
                                    const uint4 u4 = philox(make_uint4(cbase, (uint32_t)s, (uint32_t)r, d.inst_id),
                                                            a.seed, 0u);
                                    int c0, c1, c2, c3;
                                    accept_cuts(u4, tl2, e0, dm1, dcut, thr, c0, c1, c2, c3);
                                    cutp[j][0] = (uint32_t)c0 | ((uint32_t)c1 << 16);
                                    cutp[j][1] = (uint32_t)c2 | ((uint32_t)c3 << 16);
                                    break;
                                }
                                const uint64_t am = ballot64(dE <= 0) & openm;
                                if (!am) {
                                    walking = false;
                                    break;
                                }
                                flip(j, am, openm);
                            }
                        }
                        if (walking) {
                            const int cut = (int)((cutp[j][ti >> 1] >> (16 * (ti & 1))) & 0xffffu);
                            const int rel = cut - dE0[j];   // accept iff k dplus < cut - dE0
                            uint64_t am = ballot64(__mul24(k, dplus(j)) < rel) & openm;
                            while (am) {
                                flip(j, am, openm);
                                am = ballot64(__mul24(k, dplus(j)) < rel) & openm;
                            }
                        }
                    }
                    bool any = false;
#pragma unroll
                    for (int j = 0; j < NJ; j++) any |= accd[j] != 0;
                    if (cold) {
                    } else if (!any) {
                        // no flip: every site was visited with its dE0
#pragma unroll
                        for (int j = 0; j < NJ; j++)
                            ndraw_lane += (64 * j + L < m && (uint32_t)(dE0[j] - 1) < (uint32_t)(dcut - 1)) ? 1u : 0u;
                    } else {
#pragma unroll
                        for (int jj = 0; jj < NJ; jj++) dY[jj] += __mul24(psg, pd[jj]);
                        // visit-time dE of every site (dE0 plus dplus per net flip before it
                        // in site order), then draws, energy, counts and the step mask
                        int nab = 0, nrb = 0;   // adds / removes in earlier chunks
#pragma unroll
                        for (int j = 0; j < NJ; j++) {
                            const uint64_t rowj = ((uint64_t)mc[2 * j + 1] << 32) | (uint64_t)mc[2 * j];
                            const uint64_t adds = accd[j] & ~rowj, rems = accd[j] & rowj;
                            const int na = nab + (int)__builtin_amdgcn_mbcnt_hi(
                                                     (uint32_t)(adds >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)adds, 0u));
                            const int nr = nrb + (int)__builtin_amdgcn_mbcnt_hi(
                                                     (uint32_t)(rems >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)rems, 0u));
                            const int dEv = dE0[j] + __mul24(na - nr, dplus(j));
                            ndraw_lane += (64 * j + L < m && (uint32_t)(dEv - 1) < (uint32_t)(dcut - 1)) ? 1u : 0u;
                            const int inA = (int)((accd[j] >> L) & 1ull);
                            Elane += inA ? dEv : 0;   // |dEv| may exceed 24 bits for large penalties
                            Cc[j] += Ops::bit(mc, j, L) ? -inA : inA;
                            Yc[j] += dY[j];
                            nab += (int)__popcll(adds);
                            nrb += (int)__popcll(rems);
                            nacc_s += (uint32_t)__popcll(accd[j]);
                        }
#pragma unroll
                        for (int j = 0; j < NJ; j++) {
                            mc[2 * j] ^= (uint32_t)accd[j];
                            mc[2 * j + 1] ^= (uint32_t)(accd[j] >> 32);
                        }
                        Ops::write(rm[jt], lt, mc, L);
                    }
#pragma unroll
                    for (int j = 0; j < NJ; j++) {
                        Yp[j] = Yc[j];
                        Yc[j] = Yn[j];
                        Yn[j] = Ynn[j];
                    }
#pragma unroll
                    for (int w = 0; w < 2 * NJ; w++) {
                        mc[w] = mn[w];
                        mn[w] = mnn[w];
                    }
                }
            nacc += nacc_s;
            if (STOP && nacc_s == 0 && !ballot64(ndraw_lane != ndl0)) frozen = true;
            if (nacc_s) {
                E += wave_sum64(Elane);
                Elane = 0;
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
        // replicas that can still change: active and not frozen, or not started yet
        if (STOP && L == 0 && active && !frozen) atomicAdd(&s_live[s & 1], 1);
        // one table row in LDS: every wave is done with row s before row s + 1
        // (prefetched into registers during the sweep) replaces it
        __syncthreads();
        const bool all_frozen = STOP && s_live[s & 1] == 0;
        if (has_next) {
            uint4 *dst = reinterpret_cast<uint4 *>(sthr);
#pragma unroll
            for (int k = 0; k < KP; k++) {
                const int i = threadIdx.x + k * nthr;
                if (i < n4_next) dst[i] = pre[k];
            }
            for (int i = threadIdx.x + KP * nthr; i < n4_next; i += nthr) dst[i] = src_next[i];
        }
        __syncthreads();
        if (all_frozen) break;   // the same for every wave of the block
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
        ndraw += (uint64_t)wave_sum64((int64_t)ndraw_lane);
        if (L == 0) {
            if (a.resume) {
                nacc += a.accepts[grep];
                ndraw += a.draws[grep];
            }
            a.final_E[grep] = E;
            a.best_E[grep] = bestE;
            a.best_sweep[grep] = bestS;
            a.accepts[grep] = nacc;
            a.draws[grep] = ndraw;
        }
    }
}


}  // namespace uavq
