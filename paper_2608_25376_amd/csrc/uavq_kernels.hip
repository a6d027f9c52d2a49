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
// Factored sweeps, one replica per wavefront: the steps are visited in order;
// for step t every lane evaluates the sites of its own cells (c = lane + 64 j)
// against the state at the step start, and a ballot finds the first accepted
// site c* in site order; the flip is applied and the walk resumes at c* + 1.
// Sites before c* were rejections under an unchanged state, and the random
// word of a site is addressed by (instance, replica, sweep, step, cell)
// rather than consumed, so the result equals the sequential sweep bit for bit.
// During the walk only R_t has changed for the remaining sites of step t, so
// each open site's dE is its start value plus k (+-2P) for a uniform count k of
// net 1s gained by the step; with the exact acceptance cut of each site's word
// (the least d whose table entry is <= the word), a test is one compare.  The
// dE each site was visited with is rebuilt at the step end (draw counts,
// energy); Y_t takes the cost rows of the flipped cells.
//
// m <= 64 (k_sweep_ylds*): lane c holds the column of cell c as a step mask,
// the travel rows Y_t and the step terms 2P R_t live in LDS per replica, and
// blocks of four steps are first evaluated speculatively against the
// block-start state, which finishes most blocks at low temperature without
// the walk.  When one replica runs per SIMD (k_sweep_ylds_pc) a second wave
// per replica computes the next sweep's random words and acceptance cuts.
// 64 < m <= 576 (the generic chunked walk k_sweep_factored*, here and in
// uavq_factored.h): lane L holds the cell masks of steps L + 1 + 64 j (bits =
// cells) and the occupation count of cells L + 64 j, and travel rows are
// rebuilt from the neighbouring steps' masks.  The block-tested sweep of the
// same classes (k_sweep_chunk*, uavq_chunk.h) is launched by default; the
// generic walk stays as the variant it is checked against.
// One row of the acceptance table lives in LDS, shared by the block's
// replicas, and so do the cost matrix D and the start-cell costs as bytes
// (m <= 384 and costs below 256; otherwise they are read as 16-bit entries
// from global memory).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "uavq_device.h"
#include "uavq_internal.h"
#include "uavq_factored.h"

namespace uavq {

// ------------------------------------------------------------------ init --
// One block per work item; every unit (replica, 4-step block tb, word w)
// draws the 32 cells of that word for steps 4 tb + 1 .. 4 tb + 4 (stream 1).
__global__ __launch_bounds__(256) void k_init_states(KArgs a) {
    if (a.resume) return;   // the working states continue a previous segment
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

template <int NJ, bool STOP>
__global__ __launch_bounds__(1024) void k_sweep_factored(KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int iter = 0;; iter++) {
        const int itx = next_item(a, iter);
        if (itx < 0) break;
        factored_item<NJ, STOP>(a, itx, smem);
    }
}

// The fourth chunk class (m <= 256) holds more state per lane than a
// 1024-thread block's register budget allows: built for at most
// kWideMaxWaves waves per block and two waves per SIMD.
template <bool STOP>
__global__ __launch_bounds__(64 * kWideMaxWaves) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_sweep_factored4(
    KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int iter = 0;; iter++) {
        const int itx = next_item(a, iter);
        if (itx < 0) break;
        factored_item<4, STOP>(a, itx, smem);
    }
}

// Classes 5 and 6 (m <= 384, fields up to 19x19 with 8-bit costs): the same
// chunked walk; the lane's step masks (up to 72 words) leave room for one wave
// per SIMD only (fully unrolled per-chunk loops keep them in registers).
template <int NJ, bool STOP>
__global__ __launch_bounds__(64 * kWideMaxWaves) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_sweep_factored_wide(
    KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int iter = 0;; iter++) {
        const int itx = next_item(a, iter);
        if (itx < 0) break;
        factored_item<NJ, STOP>(a, itx, smem);
    }
}


// ------------------------------------------------ sweep, LDS-resident rows --
// Variant for m <= 64 (one cell per lane): lane c keeps its cell's column of
// the state as a 64-bit step mask, and the travel rows Y_t (t = 1..m) are
// kept in LDS (int16, one 64-entry row per step) and updated on accepts, so
// that visiting a step costs one LDS read (issued a step ahead) and a ballot.
// Same trajectory as k_sweep_factored bit for bit.
//
// PC (producer/consumer): the block holds two waves per replica.  The random
// words, and so the acceptance cuts, depend only on (site, sweep, replica),
// not on the state, so the second wave (the producer) computes the cuts of
// every site for sweep s+1 (Philox + the exact cut search against table row
// s+1) while the first (the consumer) sweeps s with the cuts it was given, at
// no cost beyond one LDS read per block; the two share a SIMD, so the
// producer's vector work fills the issue slots the consumer's latency-bound
// walk leaves idle.  The producer works for sweep s+1 only if sweep s-1 had a
// draw; without cuts the consumer draws for itself, reading the table row from
// global memory (the LDS row is the producer's).
template <bool PC, bool STOP>
__device__ __forceinline__ void ylds_item(const KArgs &a, int itx, uint8_t *smem) {
    constexpr int KP = 6;
    const WorkItem it = a.items[itx];
    const InstDesc d = a.desc[it.inst];
    const int m = d.m, W = d.row_words, twoP = 2 * d.P;
    const int wave = threadIdx.x >> 6, L = threadIdx.x & 63;
    const int nthr = blockDim.x, nwaves = nthr >> 6;
    const int ncons = PC ? nwaves >> 1 : nwaves;    // replica slots (consumer waves)
    const bool producer = PC && wave >= ncons;
    const int slot = producer ? wave - ncons : wave;
    const int NB = (m + 3) >> 2;                    // blocks of four steps
    const int Ts = a.thr_stride;
    // this instance's schedule: sweep s reads table row sched_row + s * sched_step
    const int srow = d.sched_row, dstep = d.sched_step;

    // LDS: the table row | D | start-cell costs | signed cost rows | per-wave travel rows
    uint32_t *sthr = reinterpret_cast<uint32_t *>(smem);
    uint8_t *sD = smem + 4 * (size_t)Ts;
    uint8_t *sdep = sD + al16((size_t)m * m);
    // sDs[(0 or m) + c][L] = +D[c][L] or -D[c][L] (int16, rows of 64, 0 for L >= m): the
    // change of Y_t when step t gains or loses cell c
    int16_t *sDs = reinterpret_cast<int16_t *>(sdep + al16((size_t)m));
    uint16_t *Yall = reinterpret_cast<uint16_t *>(sDs + 2 * 64 * (size_t)m);
    uint16_t *Yw = Yall + (size_t)slot * 64 * (m + 8);   // Y_t[c] at Yw[(t-1)*64 + c], t = 1..m+8
    // per slot, 2P R_t for t = 1..m at index t-1 (68 entries: blocks read four at a time, 0 past m)
    int *Rall = reinterpret_cast<int *>(smem + al16(reinterpret_cast<uint8_t *>(Yall + (size_t)ncons * 64 * (m + 8)) - smem));
    int *Rw = Rall + (size_t)slot * 68;
    // PC: per slot, cuts of two sweeps (by parity) [2][NB][64] as four uint16
    // per lane and block, then per slot and parity the flags "cuts valid" and
    // "the sweep had a draw"
    uint2 *cutbuf = reinterpret_cast<uint2 *>(Rall + (size_t)ncons * 68);
    int *pc_valid = reinterpret_cast<int *>(cutbuf + (size_t)ncons * 2 * NB * 64);
    int *pc_drew = pc_valid + 2 * ncons;
    __shared__ int s_first_sh;
    __shared__ int s_live[2];   // replicas of the block that can still change, by sweep parity

    {
        const uint4 *gD = reinterpret_cast<const uint4 *>(a.ws + d.d_off);
        const uint4 *gdep = reinterpret_cast<const uint4 *>(a.ws + d.ddep_off);
        const int nD4 = (m * m + 15) >> 4, nd4 = (m + 15) >> 4;
        for (int i = threadIdx.x; i < nD4; i += nthr) reinterpret_cast<uint4 *>(sD)[i] = gD[i];
        for (int i = threadIdx.x; i < nd4; i += nthr) reinterpret_cast<uint4 *>(sdep)[i] = gdep[i];
        const uint8_t *gDb = a.ws + d.d_off;
        for (int i = threadIdx.x; i < 2 * 64 * m; i += nthr) {
            const int c = (i >> 6) % m, l = i & 63;
            const int v = l < m ? (int)gDb[c * m + l] : 0;
            sDs[i] = (int16_t)(i < 64 * m ? v : -v);
        }
    }
    const bool active = slot < it.nrep;
    const int r = it.rep0 + slot;
    const int64_t grep = d.rep_base + r;
    const int s0 = active ? max(a.start_sweep ? a.start_sweep[grep] : 0, a.s_begin) : a.s_end;
    if (threadIdx.x == 0) {
        s_first_sh = a.s_end;
        if (STOP) s_live[0] = s_live[1] = 0;
    }
    if (PC && producer && L < 2) {
        pc_valid[2 * slot + L] = 0;   // no cuts yet
        pc_drew[2 * slot + L] = 1;    // no history: produce
    }
    __syncthreads();
    if (L == 0) atomicMin(&s_first_sh, s0);
    __syncthreads();
    const int s_first = s_first_sh;
    // the LDS table row: row s (row s+1, the producer's, with PC)
    const int s_row0 = PC ? s_first + 1 : s_first;
    if (s_row0 < a.s_end) {
        const int n4 = (uniform_load(a.dcut, srow + s_row0 * dstep) + 2 + 3) >> 2;   // through index dcut + 1
        const uint4 *src = reinterpret_cast<const uint4 *>(a.thr + (size_t)(srow + s_row0 * dstep) * Ts);
        uint4 *dst = reinterpret_cast<uint4 *>(sthr);
        for (int i = threadIdx.x; i < n4; i += nthr) dst[i] = src[i];
    }
    __syncthreads();

    const bool lane_in = L < m;
    const uint64_t lanes_m = m >= 64 ? ~0ull : ((1ull << m) - 1ull);
    const int dep = lane_in ? (int)sdep[L] : 0;
    uint32_t *st = a.states + d.state_off + (int64_t)r * d.state_words;

    // ---- initial state: rows (lane L holds step L+1) -> columns, counts, travel rows, energy
    uint64_t cm = 0;      // bit t-1: x_{t, L}
    int Cc = 0;
    int64_t E = 0;
    if (active && !producer) {
        uint32_t rw0 = 0u, rw1 = 0u;
        if (lane_in) {
            rw0 = st[L * W];
            if (W > 1) rw1 = st[L * W + 1];
            if (!a.resume) {   // the best state starts as the initial state
                uint32_t *bs = a.best_states + d.state_off + (int64_t)r * d.state_words;
                bs[L * W] = rw0;
                if (W > 1) bs[L * W + 1] = rw1;
            }
        }
        int64_t lane_e = 0, rowterm = 0;
        int Yp = dep;
        for (int t = 1; t <= m; t++) {
            const uint32_t r0 = __builtin_amdgcn_readlane(rw0, t - 1);
            const uint32_t r1 = __builtin_amdgcn_readlane(rw1, t - 1);
            const uint64_t row = ((uint64_t)r1 << 32) | r0;
            const int x = lane_in ? (int)((row >> L) & 1ull) : 0;
            cm |= (uint64_t)x << (t - 1);
            Cc += x;
            const int R = __popcll(row);
            if (L == 0) Rw[t - 1] = twoP * R;
            rowterm += (int64_t)d.P * R * (R - 1) - (int64_t)twoP * R;
            lane_e += x * Yp;
            if (t == m && d.closed) lane_e += x * dep;
            int Yt = 0;
            uint64_t bits = row;
            while (bits) {
                const int b = __builtin_ctzll(bits);
                bits &= bits - 1ull;
                if (lane_in) Yt += sD[b * m + L];
            }
            Yw[(t - 1) * 64 + L] = (uint16_t)Yt;
            Yp = Yt;
        }
        lane_e += (int64_t)d.P * Cc * (Cc - 1);
        E = d.c0 + rowterm + wave_sum64(lane_e);
        // boundary rows: step m+1 is the return leg (start-cell costs, or 0 for
        // an open path), steps beyond it are zero; reads past m need no test
        for (int t = m + 1; t <= m + 8; t++) Yw[(t - 1) * 64 + L] = (uint16_t)(t == m + 1 && d.closed ? dep : 0);
        if (L == 0)
            for (int t = m + 1; t <= 68; t++) Rw[t - 1] = 0;
    }

    // best so far and counters: fresh, or those of the previous segment
    int64_t bestE = LLONG_MAX;
    int bestS = -1;
    uint64_t bestcm = cm;
    bool improved = false;      // the best state changed in this launch
    int Kc = twoP * (Cc - 1);   // 2P (C_c - 1): the cell-count part of the field
    uint64_t nacc = 0, ndraw = 0;   // this launch's counts (a resumed run adds the stored ones at the end)
    if (active && a.resume) {
        bestE = a.best_E[grep];
        bestS = a.best_sweep[grep];
    }
    int64_t Elane = 0;         // energy change of the lane's accepted flips in the current sweep
    uint32_t ndraw_lane = 0;   // draws of the lane's sites visited by the sequential walk
    bool frozen = false;       // stop_frozen: a sweep had neither an accept nor a draw

    for (int s = s_first; s < a.s_end; s++) {
        uint4 pre[KP];
        const int s_pre = PC ? s + 2 : s + 1;   // the row the LDS table holds next
        const bool has_next = s_pre < a.s_end;
        const int n4_next = has_next ? (uniform_load(a.dcut, srow + s_pre * dstep) + 2 + 3) >> 2 : 0;
        const uint4 *src_next = reinterpret_cast<const uint4 *>(a.thr + (size_t)(srow + s_pre * dstep) * Ts);
#pragma unroll
        for (int k = 0; k < KP; k++) {
            const int i = threadIdx.x + k * nthr;
            pre[k] = has_next ? src_next[i < n4_next ? i : 0] : make_uint4(0u, 0u, 0u, 0u);
        }
        // with PC the consumer's own draws read row s from global memory
        const uint32_t *thr = PC ? a.thr + (size_t)(srow + s * dstep) * Ts : sthr;
        const int dcut = uniform_load(a.dcut, srow + s * dstep);
        const float tl2 = __builtin_amdgcn_exp2f(d.tl2_a + d.tl2_b * (float)s);   // ~ T_s ln 2
        const float e0 = 32.0f * tl2 - 0.5f, dm1 = (float)(dcut - 1);
        if (STOP && threadIdx.x == 0) s_live[(s + 1) & 1] = 0;   // its last reader passed the previous sweep's barriers
        if (PC && producer) {
            // cuts of every site for sweep s+1 (table row s+1 is in LDS)
            const int sp = s + 1;
            const bool prod = active && sp < a.s_end && sp >= s0 && pc_drew[2 * slot + ((s - 1) & 1)] != 0;
            if (L == 0) pc_valid[2 * slot + (sp & 1)] = prod ? 1 : 0;
            if (prod) {
                const int dcut_p = uniform_load(a.dcut, srow + sp * dstep);
                const float tl2p = __builtin_amdgcn_exp2f(d.tl2_a + d.tl2_b * (float)sp);
                const float e0p = 32.0f * tl2p - 0.5f, dm1p = (float)(dcut_p - 1);
                uint2 *cb = cutbuf + (size_t)(2 * slot + (sp & 1)) * NB * 64 + L;
                for (int b = 0; b < NB; b++) {
                    const uint4 u4 = philox(make_uint4((uint32_t)L + 65536u * (uint32_t)b, (uint32_t)sp, (uint32_t)r,
                                                       d.inst_id), a.seed, 0u);
                    int c0, c1, c2, c3;
                    accept_cuts(u4, tl2p, e0p, dm1p, dcut_p, sthr, c0, c1, c2, c3);
                    cb[b * 64] = make_uint2((uint32_t)c0 | ((uint32_t)c1 << 16), (uint32_t)c2 | ((uint32_t)c3 << 16));
                }
            }
        } else if (active && s >= s0 && !frozen) {
            // PC: cuts for this sweep from the producer, if it made them
            const bool cv = PC && pc_valid[2 * slot + (s & 1)] != 0;
            const uint2 *cbs = cutbuf + (size_t)(2 * slot + (s & 1)) * NB * 64 + L;
            uint2 cwn = PC ? cbs[0] : make_uint2(0u, 0u);   // the next block's cuts, read a block ahead
            int4 cqn = *reinterpret_cast<const int4 *>(Rw);   // the next block's 2P R_t
            const uint32_t ndl0 = ndraw_lane;
            // Steps are visited in blocks of four (the Philox blocks); Yv[k] holds
            // Y_{t0-1+k} for the block starting at step t0, and the travel rows of
            // the next block are prefetched from LDS while this one is processed.
            int Yv0 = dep;                       // Y_{t0-1}, final
            int Yv1 = Yw[L];                     // Y_{t0}
            int pf[4];
#pragma unroll
            for (int k = 0; k < 4; k++) pf[k] = Yw[(1 + k) * 64 + L];   // steps 2..5 (padded)
            uint32_t nacc_s = 0, ndraw_s = 0;
            bool spec = true;
            for (int t0 = 1; t0 <= m; t0 += 4) {
                int Yv[6];
                Yv[0] = Yv0;
                Yv[1] = Yv1;
#pragma unroll
                for (int k = 0; k < 4; k++) Yv[2 + k] = pf[k];
#pragma unroll
                for (int k = 0; k < 4; k++) pf[k] = Yw[(t0 + 4 + k) * 64 + L];   // steps t0+5.. (padded)
                // the producer's cuts of this block's four steps (PC)
                uint2 cw = cwn;
                if (PC) cwn = cbs[min(((t0 - 1) >> 2) + 1, NB - 1) * 64];
                const int4 cq = cqn;
                cqn = *reinterpret_cast<const int4 *>(Rw + t0 + 3);
                const int cqa[4] = {cq.x, cq.y, cq.z, cq.w};
                bool have_ct = cv;
                // without the producer's cuts, draw them here (kept out of line: rare)
                auto need_cuts = [&]() {
                    if (!have_ct) {
                        cw = draw_cuts((uint32_t)L + 65536u * (uint32_t)((t0 - 1) >> 2), (uint32_t)s, (uint32_t)r,
                                       d.inst_id, a.seed, tl2, e0, dm1, dcut, thr);
                        have_ct = true;
                    }
                };
                bool have_u = false;
                uint4 u4 = make_uint4(0u, 0u, 0u, 0u);
                // Speculative pass: every step of the block evaluated against the
                // state at the block start (four independent chains of work).  If
                // no site of the block accepts, the block is finished here exactly
                // as the sequential sweep would finish it (the state never changed);
                // otherwise it is swept sequentially from its first step.
                bool done = false;
                if (spec && t0 + 3 <= m) {
                    // four independent evaluations, staged side by side with no
                    // branches between them: dE = A + 2P R_t for x = 0 and
                    // 4P - 2P R_t - A for x = 1, A = Y_{t-1} + Y_{t+1} + 2P (C_c - 1)
                    const uint32_t xbits = (uint32_t)(cm >> (t0 - 1));
                    bool xb[4];
                    int A[4], dEs[4];
#pragma unroll
                    for (int i = 0; i < 4; i++) xb[i] = (xbits >> i) & 1u;
#pragma unroll
                    for (int i = 0; i < 4; i++) A[i] = Yv[i] + Yv[i + 2] + Kc;
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        const int c1 = cqa[i];
                        dEs[i] = xb[i] ? (2 * twoP - c1) - A[i] : A[i] + c1;
                    }
                    const int mn = min(min(dEs[0], dEs[1]), min(dEs[2], dEs[3]));
                    if (!(ballot64(mn < dcut) & lanes_m)) {
                        done = true;                 // nothing below the cut: all rejected, no draw
                    } else if (PC) {
                        // exact cuts at hand: the block is finished if no site is below its cut
                        // (then every dE >= cut >= 1, and those below dcut drew)
                        need_cuts();
                        const int ct0 = (int)(cw.x & 0xffffu), ct1 = (int)(cw.x >> 16);
                        const int ct2 = (int)(cw.y & 0xffffu), ct3 = (int)(cw.y >> 16);
                        const bool acc = lane_in & ((dEs[0] < ct0) | (dEs[1] < ct1) | (dEs[2] < ct2) | (dEs[3] < ct3));
                        if (!ballot64(acc)) {
                            done = true;
                            const bool n0 = lane_in && dEs[0] < dcut, n1 = lane_in && dEs[1] < dcut;
                            const bool n2 = lane_in && dEs[2] < dcut, n3 = lane_in && dEs[3] < dcut;
                            ndraw_s += (uint32_t)(__popcll(ballot64(n0)) + __popcll(ballot64(n1)) +
                                                  __popcll(ballot64(n2)) + __popcll(ballot64(n3)));
                        }
                    } else if (!(ballot64(mn <= 0) & lanes_m)) {
                        // only draws: take them all; the block is finished if none accepts
                        uint32_t cbase = (uint32_t)L + 65536u * (uint32_t)((t0 - 1) >> 2);
                        asm volatile("" : "+v"(cbase));   // generator stays inside this branch
                        u4 = philox(make_uint4(cbase, (uint32_t)s, (uint32_t)r, d.inst_id), a.seed, 0u);
                        have_u = true;
                        const bool n0 = lane_in && dEs[0] < dcut, n1 = lane_in && dEs[1] < dcut;
                        const bool n2 = lane_in && dEs[2] < dcut, n3 = lane_in && dEs[3] < dcut;
                        // unconditional reads (index 0 where no draw happens) issue together
                        const uint32_t r0 = thr[n0 ? dEs[0] : 0], r1 = thr[n1 ? dEs[1] : 0];
                        const uint32_t r2 = thr[n2 ? dEs[2] : 0], r3 = thr[n3 ? dEs[3] : 0];
                        const bool acc = (n0 & (u4.x < r0)) | (n1 & (u4.y < r1)) | (n2 & (u4.z < r2)) |
                                         (n3 & (u4.w < r3));
                        if (!ballot64(acc)) {
                            done = true;
                            ndraw_s += (uint32_t)(__popcll(ballot64(n0)) + __popcll(ballot64(n1)) +
                                                  __popcll(ballot64(n2)) + __popcll(ballot64(n3)));
                        }
                    }
                }
                const uint32_t acc_before = nacc_s;
                if (!done) {
                    // Sequential walk.  Until a site of the block needs a draw the
                    // cut is 1 (accept iff dE <= 0); from then on the exact cuts of
                    // the block's four steps make every acceptance test one compare.
                    // Its chain of dependent ballots issues first on the SIMD (without
                    // the producer: the other waves' speculative passes fill the gaps).
                    if (!PC) __builtin_amdgcn_s_setprio(2);
                    bool have_cut = PC;   // PC: always the exact cuts
                    int cut0 = 1, cut1 = 1, cut2 = 1, cut3 = 1;
                    if (PC) {
                        need_cuts();
                        cut0 = (int)(cw.x & 0xffffu);
                        cut1 = (int)(cw.x >> 16);
                        cut2 = (int)(cw.y & 0xffffu);
                        cut3 = (int)(cw.y >> 16);
                    }
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        const int t = t0 + i;
                        if (t > m) break;
                        const bool xb = (cm >> (t - 1)) & 1ull;
                        const uint64_t rmask = ballot64(xb);
                        const int h = Yv[i] + Yv[i + 2] + Kc - (xb ? 2 * twoP : 0) + cqa[i];
                        const int dE0 = xb ? -h : h;            // dE against the state at the step start
                        const int dplus = xb ? -twoP : twoP;    // change of dE per net 1 gained by step t
                        uint64_t openm = lanes_m, accd = 0;
                        int k = 0;                              // net 1s gained by step t so far
                        int dY = 0, pdv = 0;                    // signed cost-row entry of the last flip, added one step late
                        // flip the first accepted site of accm
                        auto flip = [&](uint64_t accm) {
                            const int cstar = __builtin_ctzll(accm);
                            accd |= 1ull << cstar;
                            dY += pdv;
                            const bool clears = (rmask >> cstar) & 1ull;   // the flip clears x_{t,c*}
                            pdv = sDs[((clears ? m : 0) + cstar) * 64 + L];
                            k += clears ? -1 : 1;
                            openm &= ~1ull << cstar;
                        };
                        bool walking = true;
                        if (!have_cut) {
                            // no exact cut yet: accept iff dE <= 0 while no open site needs a draw
                            while (true) {
                                const int dE = dE0 + __mul24(k, dplus);
                                if (ballot64((uint32_t)(dE - 1) < (uint32_t)(dcut - 1)) & openm) {
                                    have_cut = true;
                                    if (!have_u) {
                                        uint32_t cbase = (uint32_t)L + 65536u * (uint32_t)((t0 - 1) >> 2);
                                        asm volatile("" : "+v"(cbase));   // generator stays inside this branch
                                        u4 = philox(make_uint4(cbase, (uint32_t)s, (uint32_t)r, d.inst_id), a.seed, 0u);
                                        have_u = true;
                                    }
                                    accept_cuts(u4, tl2, e0, dm1, dcut, thr, cut0, cut1, cut2, cut3);
                                    break;
                                }
                                const uint64_t accm = ballot64(dE <= 0) & openm;
                                if (!accm) {
                                    walking = false;
                                    break;
                                }
                                flip(accm);
                            }
                        }
                        if (walking) {
                            const int cut = i == 0 ? cut0 : (i == 1 ? cut1 : (i == 2 ? cut2 : cut3));
                            const int rel = cut - dE0;          // accept iff k dplus < cut - dE0
                            uint64_t accm = ballot64(__mul24(k, dplus) < rel) & openm;
                            while (accm) {
                                flip(accm);
                                accm = ballot64(__mul24(k, dplus) < rel) & openm;
                            }
                        }
                        dY += pdv;
                        // the dE each site was visited with: dE0 plus dplus per net flip before it
                        int dEv = dE0;
                        if (accd) {
                            const uint64_t adds = accd & ~rmask, rems = accd & rmask;
                            const int na = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(adds >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)adds, 0u));
                            const int nr = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(rems >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)rems, 0u));
                            dEv = dE0 + __mul24(na - nr, dplus);
                        }
                        // draws of this step, counted per lane (lanes >= m are dropped at the end)
                        ndraw_lane += (uint32_t)(dEv - 1) < (uint32_t)(dcut - 1) ? 1u : 0u;
                        if (accd) {
                            if (L == 0) Rw[t - 1] = twoP * (int)__popcll(rmask ^ accd);   // the step's new R_t
                            nacc_s += (uint32_t)__popcll(accd);
                            const int inA = (int)((accd >> L) & 1ull);   // this lane's site was flipped
                            cm ^= (uint64_t)inA << (t - 1);
                            Kc += __mul24(inA, dplus);
                            Elane += inA ? dEv : 0;   // |dEv| may exceed 24 bits for large penalties
                            Yv[i + 1] += dY;
                        }
                    }
                    // travel rows of the walked block, for the next sweep's reads
#pragma unroll
                    for (int i = 0; i < 4; i++)
                        if (t0 + i <= m) Yw[(t0 + i - 1) * 64 + L] = (uint16_t)Yv[i + 1];
                    if (!PC) __builtin_amdgcn_s_setprio(0);
                }
                Yv0 = Yv[4];
                Yv1 = Yv[5];
                // speculate on the next block only after a block without accepted flips
                spec = nacc_s == acc_before;
            }
            nacc += nacc_s;
            ndraw += ndraw_s;
            const bool drew = ndraw_s != 0 || (ballot64(ndraw_lane != ndl0) & lanes_m) != 0;
            // tell the producer whether this sweep drew (it then makes the cuts of sweep s+2)
            if (PC && L == 0) pc_drew[2 * slot + (s & 1)] = drew ? 1 : 0;
            if (STOP && nacc_s == 0 && !drew) frozen = true;
            if (nacc_s) {
                E += wave_sum64(Elane);
                Elane = 0;
            }
            if (E < bestE) {
                bestE = E;
                bestS = s;
                bestcm = cm;
                improved = true;
            }
        }
        // replicas that can still change: active and not frozen, or not started yet
        if (STOP && L == 0 && !producer && active && !frozen) atomicAdd(&s_live[s & 1], 1);
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

    if (active && !producer) {
        // columns -> rows for the final and best states
        uint32_t f0 = 0u, f1 = 0u, b0 = 0u, b1 = 0u;
        for (int t = 1; t <= m; t++) {
            const uint64_t fr = ballot64((cm >> (t - 1)) & 1ull);
            const uint64_t br = ballot64((bestcm >> (t - 1)) & 1ull);
            if (L == t - 1) {
                f0 = (uint32_t)fr;
                f1 = (uint32_t)(fr >> 32);
                b0 = (uint32_t)br;
                b1 = (uint32_t)(br >> 32);
            }
        }
        if (lane_in) {
            st[L * W] = f0;
            if (W > 1) st[L * W + 1] = f1;
            if (improved) {
                uint32_t *bs = a.best_states + d.state_off + (int64_t)r * d.state_words;
                bs[L * W] = b0;
                if (W > 1) bs[L * W + 1] = b1;
            }
        }
        ndraw += (uint64_t)wave_sum64(lane_in ? (int64_t)ndraw_lane : 0);
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

template <bool STOP>
__global__ __launch_bounds__(1024) void k_sweep_ylds(KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int iter = 0;; iter++) {
        const int itx = next_item(a, iter);
        if (itx < 0) break;
        ylds_item<false, STOP>(a, itx, smem);
    }
}

// Same sweep for launches that hold at most one wave per SIMD: each replica's
// walk is a latency-bound chain, so with no other wave to switch to the
// compiler may spend registers on overlapping independent work instead.
template <bool STOP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_sweep_ylds_w1(KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int iter = 0;; iter++) {
        const int itx = next_item(a, iter);
        if (itx < 0) break;
        ylds_item<false, STOP>(a, itx, smem);
    }
}

// The same launch shape with a cut-producing wave beside each replica's wave
// (two waves per SIMD).
template <bool STOP>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_sweep_ylds_pc(KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    for (int iter = 0;; iter++) {
        const int itx = next_item(a, iter);
        if (itx < 0) break;
        ylds_item<true, STOP>(a, itx, smem);
    }
}

__global__ void k_fill_i32(int32_t *p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
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

// Per replica: N attempts for every sweep it ran in this launch (sweeps
// max(start_sweep, s_begin) .. s_end-1), added to the carried count on resume.
__global__ __launch_bounds__(256) void k_count_attempts(KArgs a) {
    const int inst = blockIdx.x;
    const InstDesc d = a.desc[inst];
    const uint64_t N = (uint64_t)d.m * (uint64_t)d.m;
    for (int r = threadIdx.x; r < d.nrep; r += blockDim.x) {
        const int64_t g = d.rep_base + r;
        const int s0 = max(a.start_sweep ? a.start_sweep[g] : 0, a.s_begin);
        const uint64_t run = a.s_end > s0 ? (uint64_t)(a.s_end - s0) : 0;
        a.attempts[g] = (a.resume ? a.attempts[g] : 0) + N * run;
    }
}

// violations[i] += (E[i] != E_check[i]): the invariant check of anneal_checked
__global__ void k_count_mismatch(const int64_t *E, const int64_t *E_check, uint32_t *violations, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) violations[i] += E[i] != E_check[i] ? 1u : 0u;
}

// ------------------------------------------------------------- launchers --
static size_t ylds_lds_bytes(const uavq_plan *pl, int m, int wpb) {
    return ylds_lds_bytes_for((size_t)pl->thr_stride, m, wpb);
}

// + the producer/consumer pairs' cut buffers (two sweeps of ceil(m/4) blocks of
// 64 uint2) and their flags
static size_t ylds_pc_lds_bytes(const uavq_plan *pl, int m, int wpb) {
    return ylds_lds_bytes(pl, m, wpb) + (size_t)wpb * 2 * ((m + 3) / 4) * 64 * 8 + (size_t)wpb * 4 * 4;
}

static size_t factored_lds_bytes(const uavq_plan *pl, int m, int cls, bool pw) {
    if (cls > kByteChunks) return 4 * (size_t)pl->thr_stride + 16;   // costs stay in global memory
    // + 64: cost-row reads of lanes past m run up to 63 bytes beyond D; + 1 KB per wave for the block-tested
    // sweep's packed draw words (two and three chunks), when asked for
    return 4 * (size_t)pl->thr_stride + al16((size_t)m * m) + al16((size_t)m) + 64 +
           (pw ? 1024 * (size_t)pl->waves_per_block[cls] : 0);
}

static int class_mmax(const uavq_plan *pl, int cls) {
    int mmax = 0;
    for (int i = pl->class_begin[cls]; i < pl->class_begin[cls + 1]; i++)
        mmax = std::max(mmax, pl->desc[pl->items[i].inst].m);
    return mmax;
}

bool ylds_fits(const uavq_plan *pl) {
    return ylds_lds_bytes(pl, class_mmax(pl, 1), pl->waves_per_block[1]) <= 160 * 1024;
}

static bool use_ylds(const uavq_plan *pl) { return pl->variant != UAVQ_VARIANT_ROWMASK && ylds_fits(pl); }

template <bool STOP>
static const void *class_kernel_t(const uavq_plan *pl, int cls) {
    if (cls == 1 && use_ylds(pl) && pl->ylds_pc) return (const void *)k_sweep_ylds_pc<STOP>;
    if (cls == 1 && use_ylds(pl))
        return pl->ylds_w1 ? (const void *)k_sweep_ylds_w1<STOP> : (const void *)k_sweep_ylds<STOP>;
    if (cls == 1) return (const void *)k_sweep_factored<1, STOP>;
    if (cls >= 2 && cls <= 4 && !pl->generic_chunk) return chunk_sweep_kernel(cls, STOP);
    if ((cls == 5 || cls == 6) && !pl->generic_chunk) return chunk_sweep_wide_kernel(cls, STOP);
    if (cls >= 7 && !pl->generic_chunk) return chunk_sweep_big_kernel(cls, STOP);
    if (cls == 2) return (const void *)k_sweep_factored<2, STOP>;
    if (cls == 3) return (const void *)k_sweep_factored<3, STOP>;
    if (cls == 4) return (const void *)k_sweep_factored4<STOP>;
    if (cls == 5) return (const void *)k_sweep_factored_wide<5, STOP>;
    if (cls == 6) return (const void *)k_sweep_factored_wide<6, STOP>;
    return big_sweep_kernel(cls, STOP);
}

static const void *class_kernel(const uavq_plan *pl, int cls) {
    return pl->stop_frozen ? class_kernel_t<true>(pl, cls) : class_kernel_t<false>(pl, cls);
}

// Kernel attributes and occupancy, once per plan and outside any stream
// capture: dynamic LDS limits and, for persistent launches, resident blocks.
static int prepare(const uavq_plan *cpl) {
    uavq_plan *pl = const_cast<uavq_plan *>(cpl);
    std::lock_guard<std::mutex> lock(pl->mu);   // the only writer of these fields after creation
    if (pl->prepared) return UAVQ_OK;
    int dev = 0;
    UAVQ_HIP(hipGetDevice(&dev));
    UAVQ_HIP(hipDeviceGetAttribute(&pl->cu_count, hipDeviceAttributeMultiprocessorCount, dev));
    {
        // one wave per SIMD when every wave of the m <= 64 launch is resident at once
        const int n1 = pl->class_begin[2] - pl->class_begin[1], w1 = pl->waves_per_block[1];
        pl->ylds_w1 = use_ylds(pl) && w1 <= 4 && (int64_t)n1 * w1 <= 4 * (int64_t)pl->cu_count;
        // and a cut-producing wave beside each replica when the pair still fits (cuts are uint16)
        pl->ylds_pc = pl->ylds_w1 && !pl->no_producer && pl->Dmax < 65535 &&
                      ylds_pc_lds_bytes(pl, class_mmax(pl, 1), w1) <= 160 * 1024;
    }
    for (int cls = 1; cls <= kMaxChunks; cls++) {
        if (pl->dense || pl->class_begin[cls + 1] <= pl->class_begin[cls]) continue;
        const int mmax = class_mmax(pl, cls), wpb = pl->waves_per_block[cls];
        const bool pc = cls == 1 && use_ylds(pl) && pl->ylds_pc;
        size_t lds = pc ? ylds_pc_lds_bytes(pl, mmax, wpb)
                        : (cls == 1 && use_ylds(pl)) ? ylds_lds_bytes(pl, mmax, wpb)
                                                     : factored_lds_bytes(pl, mmax, cls, false);
        if (lds > 160 * 1024)
            return set_error(UAVQ_ETOOBIG, "anneal: LDS need %zu bytes (m = %d, Dmax = %d)", lds, mmax, pl->Dmax);
        const void *k = class_kernel(pl, cls);
        UAVQ_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        int nb = 0;
        UAVQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, (pc ? 128 : 64) * wpb, lds));
        pl->pw_class[cls] = 0;
        if (cls >= 2 && cls <= 3 && !pl->generic_chunk) {
            // the packed draw words' LDS only where it leaves the resident workgroups per CU as they are
            const size_t lds_pw = factored_lds_bytes(pl, mmax, cls, true);
            int nb_pw = 0;
            if (lds_pw <= 160 * 1024) {
                UAVQ_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_pw));
                UAVQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb_pw, k, 64 * wpb, lds_pw));
            }
            if (nb_pw >= nb) {
                lds = lds_pw;
                pl->pw_class[cls] = 1;
            } else {
                UAVQ_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            }
        }
        pl->max_blocks[cls] = std::max(nb, 1);
        pl->lds_class[cls] = lds;
    }
    if (pl->concurrent && !pl->dense) {
        // one stream per class after the first (default priority), fork/join events
        int used = 0;
        for (int cls = 1; cls <= kMaxChunks; cls++) {
            if (pl->class_begin[cls + 1] <= pl->class_begin[cls]) continue;
            if (used++ == 0) continue;
            hipStream_t s2;
            hipEvent_t e2;
            UAVQ_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
            pl->side_stream[cls] = (void *)s2;
            UAVQ_HIP(hipEventCreateWithFlags(&e2, hipEventDisableTiming));
            pl->join_ev[cls] = (void *)e2;
        }
        if (used > 1) {
            hipEvent_t e;
            UAVQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            pl->fork_ev = (void *)e;
        }
    }
    pl->prepared = 1;
    return UAVQ_OK;
}

static int launch_class(const uavq_plan *pl, KArgs a, int cls, hipStream_t st) {
    const int b0 = pl->class_begin[cls], b1 = pl->class_begin[cls + 1];
    if (b1 <= b0) return UAVQ_OK;
    const int n = b1 - b0, wpb = pl->waves_per_block[cls];
    a.item_base = b0;
    int grid = n;
    if (pl->persistent) {
        a.queue = (int32_t *)(a.ws + pl->queue_off) + cls;
        a.queue_n = n;
        grid = std::min(n, pl->max_blocks[cls] * pl->cu_count);
    } else {
        a.queue = nullptr;
        a.queue_n = 0;
    }
    const bool timed = pl->timing && !pl->graph;
    if (timed) UAVQ_HIP(hipEventRecord((hipEvent_t)pl->ev[2 * cls], st));
    const size_t lds = pl->lds_class[cls];
    a.pw = pl->pw_class[cls];
    const void *kern = class_kernel(pl, cls);
    const int threads = (cls == 1 && use_ylds(pl) && pl->ylds_pc ? 128 : 64) * wpb;
    void *kargs[] = {&a};
    UAVQ_HIP(hipLaunchKernel(kern, dim3(grid), dim3(threads), kargs, lds, st));
    UAVQ_HIP(hipGetLastError());
    if (timed) UAVQ_HIP(hipEventRecord((hipEvent_t)pl->ev[2 * cls + 1], st));
    return UAVQ_OK;
}

// energies of the final states recomputed by the MFMA refresh (invariant check)
static int launch_checks(const uavq_plan *pl, const KArgs &a, int64_t *check_E, hipStream_t st) {
    for (int i = 0; i < pl->n_inst; i++) {
        const InstDesc &d = pl->desc[i];
        if (d.wide || d.chunks > kByteChunks)
            return set_error(UAVQ_ETOOBIG, "energy check: instance %d has costs above 255 or m = %d > %d", i, d.m,
                             64 * kByteChunks);
        int rc = launch_energy_refresh(a.states + d.state_off, d.nrep, check_E + d.rep_base, a.ws + d.d_off,
                                       a.ws + d.ddep_off, d.m, d.P, d.closed, d.c0, st);
        if (rc) return rc;
    }
    return UAVQ_OK;
}

// init -> sweeps (one kernel per chunk class) -> reduce [-> energy check]
int launch_anneal(const uavq_plan *pl, const KArgs &a0, void *stream, int64_t *check_E) {
    hipStream_t st = (hipStream_t)stream;
    KArgs a = a0;
    const int n_items = (int)pl->items.size();
    if (n_items == 0) return UAVQ_OK;
    a.item_base = 0;
    a.queue = nullptr;
    if (!a.resume) {   // a resumed segment continues the working states
        hipLaunchKernelGGL(k_init_states, dim3(n_items), dim3(256), 0, st, a);
        UAVQ_HIP(hipGetLastError());
    }
    int rc;
    if (pl->dense) {
        if ((rc = launch_dense(pl, a, st))) return rc;
    } else {
        if (pl->persistent) {
            // reset the item counters with a kernel (graph-safe, no memset node)
            hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, (int32_t *)(a.ws + pl->queue_off), kMaxChunks + 2, 0);
            UAVQ_HIP(hipGetLastError());
        }
        if (pl->fork_ev) {
            // classes at the same time: the first on st, the others on the plan's streams
            const bool timed = pl->timing && !pl->graph;
            if (timed) UAVQ_HIP(hipEventRecord((hipEvent_t)pl->ev[0], st));
            UAVQ_HIP(hipEventRecord((hipEvent_t)pl->fork_ev, st));
            for (int cls = 1; cls <= kMaxChunks; cls++) {
                if (!pl->side_stream[cls]) {
                    if ((rc = launch_class(pl, a, cls, st))) return rc;
                    continue;
                }
                hipStream_t s2 = (hipStream_t)pl->side_stream[cls];
                UAVQ_HIP(hipStreamWaitEvent(s2, (hipEvent_t)pl->fork_ev, 0));
                if ((rc = launch_class(pl, a, cls, s2))) return rc;
                UAVQ_HIP(hipEventRecord((hipEvent_t)pl->join_ev[cls], s2));
                UAVQ_HIP(hipStreamWaitEvent(st, (hipEvent_t)pl->join_ev[cls], 0));
            }
            if (timed) UAVQ_HIP(hipEventRecord((hipEvent_t)pl->ev[1], st));
        } else {
            for (int cls = 1; cls <= kMaxChunks; cls++)
                if ((rc = launch_class(pl, a, cls, st))) return rc;
        }
    }
    if (!pl->reduce_at_end || a.s_end == pl->S) {
        hipLaunchKernelGGL(k_reduce, dim3(pl->n_inst), dim3(256), 0, st, a);
        UAVQ_HIP(hipGetLastError());
    }
    if (a.attempts) {
        hipLaunchKernelGGL(k_count_attempts, dim3(pl->n_inst), dim3(256), 0, st, a);
        UAVQ_HIP(hipGetLastError());
    }
    return check_E ? launch_checks(pl, a, check_E, st) : UAVQ_OK;
}

size_t energy_ws_bytes(const uavq_qubo *q) {
    return q ? ((size_t)q->m * q->m + 255) / 256 * 256 + ((size_t)q->m + 255) / 256 * 256 : 0;
}

int launch_energy(const uavq_qubo *q, const uint32_t *d_x, int64_t n, int64_t *d_E, void *d_ws, size_t ws_bytes,
                  void *stream) {
    if (q->D.empty()) return set_error(UAVQ_ETOOBIG, "energy_eval_dev: costs above 255 (w_max = %d)", q->wmax);
    if (!d_ws || ws_bytes < energy_ws_bytes(q)) return set_error(UAVQ_EINVAL, "energy_eval_dev: workspace too small");
    hipStream_t st = (hipStream_t)stream;
    uint8_t *dD = (uint8_t *)d_ws;
    uint8_t *ddep = dD + ((size_t)q->m * q->m + 255) / 256 * 256;
    UAVQ_HIP(hipMemcpyAsync(dD, q->D.data(), q->D.size(), hipMemcpyHostToDevice, st));
    UAVQ_HIP(hipMemcpyAsync(ddep, q->ddep.data(), q->ddep.size(), hipMemcpyHostToDevice, st));
    return launch_energy_refresh(d_x, n, d_E, dD, ddep, q->m, q->P, q->closed, q->c0, st);
}

static uint64_t mix64(uint64_t h, uint64_t v) {
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h;
}

static void release_graph(uavq_plan *pl) {
    if (pl->graph_exec) {
        (void)hipGraphExecDestroy((hipGraphExec_t)pl->graph_exec);
        pl->graph_exec = nullptr;
        pl->graph_key = 0;
    }
}

}  // namespace uavq

using namespace uavq;

extern "C" {

int uavq_plan_upload(const uavq_plan *pl, void *d_ws, size_t ws_bytes, void *stream) {
    if (!pl || !d_ws) return set_error(UAVQ_EINVAL, "plan_upload: null argument");
    if (ws_bytes < pl->ws_bytes) return set_error(UAVQ_EINVAL, "plan_upload: workspace %zu < %zu bytes", ws_bytes, pl->ws_bytes);
    int rc = prepare(pl);
    if (rc) return rc;
    UAVQ_HIP(hipMemcpyAsync(d_ws, pl->blob.data(), pl->blob.size(), hipMemcpyHostToDevice, (hipStream_t)stream));
    return UAVQ_OK;
}

const char *uavq_plan_kernel_name(const uavq_plan *pl, int32_t cls) {
    if (!pl || cls < 1 || cls > uavq::kMaxChunks) {
        set_error(UAVQ_EINVAL, "plan_kernel_name: bad argument");
        return nullptr;
    }
    if (pl->dense) return pl->n_inst > 0 && cls == 1 ? "k_sweep_dense" : "";
    if (pl->class_begin[cls + 1] <= pl->class_begin[cls]) return "";
    if (uavq::prepare(pl)) return nullptr;   // the one-wave choice needs the device's CU count
    if (cls == 1 && uavq::use_ylds(pl) && pl->ylds_pc) return "k_sweep_ylds_pc";
    if (cls == 1 && uavq::use_ylds(pl)) return pl->ylds_w1 ? "k_sweep_ylds_w1" : "k_sweep_ylds";
    if (cls == 2 && !pl->generic_chunk) return "k_sweep_chunk<2>";
    if (cls == 3 && !pl->generic_chunk) return "k_sweep_chunk<3>";
    if (cls == 4 && !pl->generic_chunk) return "k_sweep_chunk<4>";
    if (cls == 5 && !pl->generic_chunk) return "k_sweep_chunk<5>";
    if (cls == 6 && !pl->generic_chunk) return "k_sweep_chunk<6>";
    if (cls == 7 && !pl->generic_chunk) return "k_sweep_chunk_big<7>";
    if (cls >= 8 && !pl->generic_chunk) return "k_sweep_chunk_big<9>";
    static const char *const names[] = {"", "k_sweep_factored<1>", "k_sweep_factored<2>", "k_sweep_factored<3>",
                                        "k_sweep_factored4", "k_sweep_factored_wide<5>", "k_sweep_factored_wide<6>",
                                        "k_sweep_factored_big<7>", "k_sweep_factored_big<9>",
                                        "k_sweep_factored_big<9>"};
    static_assert(sizeof(names) / sizeof(names[0]) == uavq::kMaxChunks + 1, "one name per chunk class");
    return names[cls];
}

int uavq_anneal_batch(const uavq_plan *pl, void *d_ws, size_t ws_bytes, const uavq_anneal_init *init,
                      const uavq_anneal_out *out, void *stream) {
    if (!pl) return set_error(UAVQ_EINVAL, "anneal_batch: null argument");
    return uavq_anneal_segment(pl, d_ws, ws_bytes, init, out, 0, pl->S, 0, stream);
}

int uavq_anneal_segment(const uavq_plan *pl, void *d_ws, size_t ws_bytes, const uavq_anneal_init *init,
                        const uavq_anneal_out *out, int32_t s_begin, int32_t s_end, int32_t resume, void *stream) {
    if (!pl || !out) return set_error(UAVQ_EINVAL, "anneal_batch: null argument");
    if (s_begin < 0 || s_end < s_begin || s_end > pl->S)
        return set_error(UAVQ_EINVAL, "anneal_segment: sweep range [%d, %d) outside [0, %d]", s_begin, s_end, pl->S);
    if (pl->total_rep == 0) return UAVQ_OK;
    if (!d_ws || ws_bytes < pl->ws_bytes) return set_error(UAVQ_EINVAL, "anneal_batch: workspace too small");
    if (!out->final_states || !out->final_E || !out->best_E || !out->best_sweep || !out->best_states ||
        !out->accepts || !out->draws)
        return set_error(UAVQ_EINVAL, "anneal_batch: a required output is NULL");
    if (init && init->seeded && !init->states)
        return set_error(UAVQ_EINVAL, "anneal_batch: seeded replicas need init->states");
    if (pl->graph && !stream) return set_error(UAVQ_EINVAL, "anneal_batch: graph mode needs a non-default stream");
    int rc = prepare(pl);
    if (rc) return rc;
    KArgs a{};
    const uint8_t *ws = (const uint8_t *)d_ws;
    a.ws = ws;
    a.desc = (const InstDesc *)(ws + pl->desc_off);
    a.items = (const WorkItem *)(ws + pl->items_off);
    a.n_items = (int32_t)pl->items.size();
    a.thr = (const uint32_t *)(ws + pl->thr_off);
    a.dcut = (const int32_t *)(ws + pl->dcut_off);
    a.S = pl->S;
    a.s_begin = s_begin;
    a.s_end = s_end;
    a.resume = resume ? 1 : 0;
    a.Dmax = pl->Dmax;
    a.thr_stride = pl->thr_stride;
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
    a.attempts = out->attempts;
    if (!pl->graph && pl->fork_ev) {
        // the plan's streams and fork/join events are shared: one launch sequence at a time
        std::lock_guard<std::mutex> lock(const_cast<uavq_plan *>(pl)->mu);
        return launch_anneal(pl, a, stream, out->check_E);
    }
    if (!pl->graph) return launch_anneal(pl, a, stream, out->check_E);

    // graph mode: replay the captured sequence while every pointer is unchanged;
    // the cached graph is shared, so capture and launch hold the plan's lock
    uavq_plan *mp = const_cast<uavq_plan *>(pl);
    std::lock_guard<std::mutex> lock(mp->mu);
    uint64_t key = 0x12345678ull;
    const void *ptrs[] = {d_ws, stream, a.init_states, a.seeded, a.start_sweep, out->final_states, out->final_E,
                          out->best_E, out->best_sweep, out->best_states, out->accepts, out->draws, out->inst_best_E,
                          out->inst_best_replica, out->inst_best_sweep, out->inst_best_state, out->check_E,
                          out->attempts};
    for (const void *p : ptrs) key = mix64(key, (uint64_t)(uintptr_t)p);
    key = mix64(mix64(mix64(key, (uint64_t)s_begin), (uint64_t)s_end), (uint64_t)a.resume);
    hipStream_t st = (hipStream_t)stream;
    if (!mp->graph_exec || mp->graph_key != key) {
        release_graph(mp);
        UAVQ_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        rc = launch_anneal(pl, a, stream, out->check_E);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return set_error(UAVQ_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        hipGraphExec_t ge = nullptr;
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return set_error(UAVQ_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        mp->graph_exec = (void *)ge;
        mp->graph_key = key;
    }
    UAVQ_HIP(hipGraphLaunch((hipGraphExec_t)mp->graph_exec, st));
    return UAVQ_OK;
}

int uavq_anneal_checked(const uavq_plan *pl, void *d_ws, size_t ws_bytes, const uavq_anneal_init *init,
                        const uavq_anneal_out *out, int32_t refresh_every, uint32_t *d_violations,
                        uint64_t *n_violations, void *stream) {
    if (!pl || !out || !n_violations || refresh_every < 1)
        return set_error(UAVQ_EINVAL, "anneal_checked: bad argument");
    *n_violations = 0;
    if (pl->total_rep == 0) return UAVQ_OK;
    if (!out->check_E || !d_violations)
        return set_error(UAVQ_EINVAL, "anneal_checked: check_E and the violation counts are required");
    if (pl->graph) return set_error(UAVQ_EINVAL, "anneal_checked: not available in graph mode");
    if (!d_ws || ws_bytes < pl->ws_bytes) return set_error(UAVQ_EINVAL, "anneal_checked: workspace too small");
    if (!out->final_states || !out->final_E || !out->best_E || !out->best_sweep || !out->best_states ||
        !out->accepts || !out->draws)
        return set_error(UAVQ_EINVAL, "anneal_checked: a required output is NULL");
    if (pl->total_rep > INT32_MAX) return set_error(UAVQ_ETOOBIG, "anneal_checked: too many replicas");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = pl->total_rep;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, st, (int32_t *)d_violations, (int)n, 0);
    UAVQ_HIP(hipGetLastError());
    for (int32_t s = 0; s < pl->S; s += refresh_every) {
        const int32_t e = (int32_t)std::min<int64_t>((int64_t)s + refresh_every, pl->S);
        int rc = uavq_anneal_segment(pl, d_ws, ws_bytes, init, out, s, e, s > 0 ? 1 : 0, stream);
        if (rc) return rc;
        hipLaunchKernelGGL(k_count_mismatch, dim3(blocks), dim3(256), 0, st, out->final_E, out->check_E,
                           d_violations, n);
        UAVQ_HIP(hipGetLastError());
    }
    std::vector<uint32_t> v((size_t)n);
    UAVQ_HIP(hipMemcpyAsync(v.data(), d_violations, v.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    UAVQ_HIP(hipStreamSynchronize(st));
    uint64_t total = 0;
    for (uint32_t x : v) total += x;
    *n_violations = total;
    if (total)
        return set_error(UAVQ_EINVARIANT, "anneal_checked: %llu pieces whose kept energy differs from the recomputed one",
                         (unsigned long long)total);
    return UAVQ_OK;
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
    if (!pl->timing || pl->graph) return set_error(UAVQ_EINVAL, "plan_sweep_ms: timing not enabled (or graph mode)");
    float total = 0.f;
    if (pl->fork_ev) {   // concurrent classes: from the fork to the join on the caller's stream
        UAVQ_HIP(hipEventElapsedTime(&total, (hipEvent_t)pl->ev[0], (hipEvent_t)pl->ev[1]));
        *ms = total;
        return UAVQ_OK;
    }
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
    release_graph(pl);
    for (int c = 0; c < kMaxChunks + 2; c++) {
        if (pl->side_stream[c]) (void)hipStreamDestroy((hipStream_t)pl->side_stream[c]);
        if (pl->join_ev[c]) (void)hipEventDestroy((hipEvent_t)pl->join_ev[c]);
        pl->side_stream[c] = pl->join_ev[c] = nullptr;
    }
    if (pl->fork_ev) (void)hipEventDestroy((hipEvent_t)pl->fork_ev);
    pl->fork_ev = nullptr;
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

// ------------------------------------------------------------- autotuner --
// Candidate launch shapes are timed with HIP events on a trial plan of
// trial_sweeps sweeps (same instances and replicas), using device memory
// allocated here; the fastest is returned and optionally cached as JSON.
static std::string tune_key(const uavq_qubo *const *q, int32_t n, const uavq_anneal_params *p, int cu) {
    int mmax[kMaxChunks + 1] = {0}, cnt[kMaxChunks + 1] = {0};
    for (int32_t i = 0; i < n; i++) {
        int c = std::min((q[i]->m + 63) / 64, kMaxChunks);
        if (q[i]->wmax > 255) c = std::max(c, kByteChunks + 1);   // 16-bit costs: the classes above bytes
        mmax[c] = std::max(mmax[c], q[i]->m);
        cnt[c]++;
    }
    char buf[256];
    int len = snprintf(buf, sizeof buf, "gfx950|cu%d|R%d|flags%u", cu, p->replicas,
                       (unsigned)(p->flags & (UAVQ_PERSISTENT | UAVQ_KERNEL_DENSE)));
    for (int c = 1; c <= kMaxChunks; c++)
        if (cnt[c]) {
            int lg = 0;
            while ((1 << (lg + 1)) <= cnt[c]) lg++;
            len += snprintf(buf + len, sizeof buf - len, "|c%d:m%d:n%d", c, (mmax[c] + 7) / 8 * 8, 1 << lg);
        }
    return std::string(buf);
}

static bool cache_lookup(const char *path, const std::string &key, uavq_tune *t) {
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char *q1 = strchr(line, '"');
        if (!q1) continue;
        char *q2 = strchr(q1 + 1, '"');
        if (!q2) continue;
        if (std::string(q1 + 1, q2) != key) continue;
        // "wpb": [one value per chunk class], "variant": u, "ms": f (a line of
        // another class count does not parse and is tuned again)
        uavq_tune v{};
        const char *w = strstr(q2 + 1, "\"wpb\": [");
        bool ok = w != nullptr;
        if (ok) w += 8;
        for (int c = 1; ok && c <= kMaxChunks; c++) {
            char *end = nullptr;
            const long x = strtol(w, &end, 10);
            ok = end != w && x >= 0 && x <= 16;
            if (!ok) break;
            v.waves_per_block[c] = (int32_t)x;
            w = end;
            if (c < kMaxChunks) ok = *w++ == ',';
        }
        unsigned var = 0;
        if (ok && sscanf(w, "], \"variant\": %u, \"ms\": %f}", &var, &v.trial_ms) == 2) {
            v.variant_flags = var;
            *t = v;
            found = true;
        }
    }
    fclose(f);
    return found;
}

static void cache_store(const char *path, const std::string &key, const uavq_tune &t) {
    std::vector<std::string> keep;
    if (FILE *f = fopen(path, "r")) {
        char line[1024];
        while (fgets(line, sizeof line, f)) {
            char *q1 = strchr(line, '"');
            if (!q1) continue;
            char *q2 = strchr(q1 + 1, '"');
            if (!q2 || std::string(q1 + 1, q2) == key) continue;
            std::string l(line);
            while (!l.empty() && (l.back() == '\n' || l.back() == ',')) l.pop_back();
            keep.push_back(l);
        }
        fclose(f);
    }
    std::string entry = "\"" + key + "\": {\"wpb\": [";
    for (int c = 1; c <= kMaxChunks; c++) entry += std::to_string(t.waves_per_block[c]) + (c < kMaxChunks ? ", " : "");
    char buf[96];
    snprintf(buf, sizeof buf, "], \"variant\": %u, \"ms\": %.4f}", (unsigned)t.variant_flags, t.trial_ms);
    keep.push_back(entry + buf);
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    for (size_t i = 0; i < keep.size(); i++) fprintf(f, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
    rename(tmp.c_str(), path);
}

int uavq_autotune(const uavq_qubo *const *q, int32_t n_inst, const uint32_t *inst_ids, const uavq_anneal_params *p,
                  int32_t trial_sweeps, const char *cache_path, uavq_tune *out) {
    if (!q || !inst_ids || !p || !out || n_inst < 1 || trial_sweeps < 1)
        return set_error(UAVQ_EINVAL, "autotune: bad argument");
    int dev = 0, cu = 0;
    UAVQ_HIP(hipGetDevice(&dev));
    UAVQ_HIP(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
    const std::string key = tune_key(q, n_inst, p, cu);
    if (cache_path && cache_lookup(cache_path, key, out)) return UAVQ_OK;

    // Chunk classes launch one after another, so each class's shape is chosen
    // on its own kernel's time (events around each class's launch); the
    // variant only concerns class 1.
    const int wpbs[] = {1, 2, 4, 8, 12, 16};   // 12: three waves per SIMD for m <= 64 where their LDS fits
    const uint32_t variants[] = {0u, UAVQ_VARIANT_ROWMASK, UAVQ_VARIANT_NOPRODUCER};
    hipStream_t st = nullptr;
    UAVQ_HIP(hipStreamCreate(&st));
    float best_cls[kMaxChunks + 1];
    int best_wpb[kMaxChunks + 1];
    uint32_t best_var = 0u;
    for (int c = 0; c <= kMaxChunks; c++) {
        best_cls[c] = 1e30f;
        best_wpb[c] = 4;
    }
    int rc = UAVQ_OK;
    for (uint32_t var : variants) {
        for (int wpb : wpbs) {
            uavq_tune t{};
            for (int c = 1; c <= kMaxChunks; c++) t.waves_per_block[c] = wpb;
            t.variant_flags = var;
            uavq_anneal_params tp = *p;
            tp.sweeps = trial_sweeps;
            // classes are timed one after another (a concurrent launch would blur their times)
            tp.flags &= ~(uint32_t)(UAVQ_GRAPH | UAVQ_VARIANT_ROWMASK | UAVQ_VARIANT_NOPRODUCER |
                                    UAVQ_CONCURRENT_CLASSES);
            tp.tune = &t;
            uavq_plan *pl = nullptr;
            if (uavq_plan_create(q, n_inst, inst_ids, &tp, &pl) != UAVQ_OK) continue;
            void *ws = nullptr, *buf = nullptr;
            const size_t R = (size_t)pl->total_rep, W = (size_t)pl->total_state_words;
            size_t inst_words = 0;
            for (int32_t i = 0; i < n_inst; i++) inst_words += (size_t)q[i]->m * q[i]->row_words;
            const size_t nbuf = 2 * W * 4 + 6 * R * 8 + n_inst * 16 + inst_words * 4 + 1024;
            bool ok = hipMalloc(&ws, pl->ws_bytes) == hipSuccess && hipMalloc(&buf, nbuf) == hipSuccess;
            float ms = 1e30f;
            if (ok && uavq_plan_upload(pl, ws, pl->ws_bytes, st) == UAVQ_OK) {
                uint8_t *b = (uint8_t *)buf;
                uavq_anneal_out o{};
                o.final_states = (uint32_t *)b;            b += W * 4;
                o.best_states = (uint32_t *)b;             b += W * 4;
                b = (uint8_t *)(((uintptr_t)b + 255) & ~(uintptr_t)255);
                o.final_E = (int64_t *)b;                  b += R * 8;
                o.best_E = (int64_t *)b;                   b += R * 8;
                o.accepts = (uint64_t *)b;                 b += R * 8;
                o.draws = (uint64_t *)b;                   b += R * 8;
                o.best_sweep = (int32_t *)b;               b += R * 8;
                o.inst_best_E = (int64_t *)b;              b += (size_t)n_inst * 8;
                o.inst_best_replica = (int32_t *)b;        b += (size_t)n_inst * 4;
                o.inst_best_sweep = (int32_t *)b;          b += (size_t)n_inst * 4;
                o.inst_best_state = (uint32_t *)b;
                float cls_ms[kMaxChunks + 1];
                for (int c = 0; c <= kMaxChunks; c++) cls_ms[c] = 1e30f;
                if (uavq_plan_set_timing(pl, 1) == UAVQ_OK &&
                    uavq_anneal_batch(pl, ws, pl->ws_bytes, nullptr, &o, st) == UAVQ_OK &&
                    hipStreamSynchronize(st) == hipSuccess) {
                    bool good = true;
                    for (int rep = 0; rep < 3 && good; rep++) {
                        good = uavq_anneal_batch(pl, ws, pl->ws_bytes, nullptr, &o, st) == UAVQ_OK &&
                               hipStreamSynchronize(st) == hipSuccess;
                        for (int c = 1; c <= kMaxChunks && good; c++) {
                            if (pl->class_begin[c + 1] <= pl->class_begin[c]) continue;
                            float e = 0.0f;
                            good = hipEventElapsedTime(&e, (hipEvent_t)pl->ev[2 * c], (hipEvent_t)pl->ev[2 * c + 1]) ==
                                   hipSuccess;
                            if (good) cls_ms[c] = std::min(cls_ms[c], e);
                        }
                    }
                    if (good) ms = 0.0f;
                }
                if (ms == 0.0f) {
                    for (int c = 1; c <= kMaxChunks; c++) {
                        if (c > 1 && var != 0u) continue;   // the variant changes class 1 only
                        if (cls_ms[c] < best_cls[c]) {
                            best_cls[c] = cls_ms[c];
                            best_wpb[c] = wpb;
                            if (c == 1) best_var = var;
                        }
                    }
                }
            }
            (void)hipStreamSynchronize(st);
            if (ws) (void)hipFree(ws);
            if (buf) (void)hipFree(buf);
            uavq_plan_free(pl);
        }
    }
    (void)hipStreamDestroy(st);
    uavq_tune best{};
    best.trial_ms = 0.0f;
    bool any = false;
    for (int c = 1; c <= kMaxChunks; c++) {
        best.waves_per_block[c] = best_wpb[c];
        if (best_cls[c] < 1e30f) {
            best.trial_ms += best_cls[c];
            any = true;
        }
    }
    best.variant_flags = best_var;
    if (!any) return set_error(UAVQ_EHIP, "autotune: no candidate ran");
    *out = best;
    if (cache_path) cache_store(cache_path, key, best);
    return rc;
}

}  // extern "C"
