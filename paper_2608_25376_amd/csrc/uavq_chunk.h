// Block-tested chunked Metropolis sweep for 64 < m <= 576 (two to nine
// 64-cell chunks per lane; the 12x12 field has m = 143), gfx950.  Built by
// uavq_sweep_chunk.hip (two to four chunks), uavq_sweep_chunk_wide.hip (five
// and six) and uavq_sweep_chunk_big.hip (seven to nine, 16-bit costs).
//
// Same trajectory as the in-order sequential sweep, bit for bit (model and
// walk: see uavq_kernels.hip).  One wavefront anneals one replica; lane L
// evaluates the cells c = 64 j + L of every step.  What differs from the
// generic chunked kernel is how a sweep spends its time when little happens:
//
//  * Step summaries.  Lane L keeps, for the steps 64 j + L + 1, the number of
//    set cells R_t and the lowest set cell p_t.  When R_t = 1 (the state is a
//    tour there) the travel row Y_t = D^T x_t is the cost row D[p_t][.]: one
//    read per chunk, no scan of the step's mask.
//  * Quiet blocks.  Steps are taken in blocks of four (the four steps that
//    share one Philox call per cell).  If every step of a block has R_t = 1,
//    the block is first evaluated against the state at its start: with no
//    site below the draw cutoff dcut (entries from dcut on are 0: rejected
//    without a draw) the block is finished -- the sequential sweep would have
//    visited every site with exactly these dE, since nothing changed; with no
//    site at dE <= 0, the block's Philox words are drawn and compared with
//    the table, and if none is accepted the block is finished too, with its
//    draws counted.  Otherwise the block is walked step by step as in the
//    generic kernel.  After a walked block with an accepted flip the next
//    block is walked directly.
//  * Selects on masks.  A step's cell mask (uniform, in scalar registers) is
//    used directly as the per-lane select condition of dE and of the +-2P
//    slope (inverse ballot), so no bit is extracted per lane.
//
// Per lane and chunk: KC_j = 2P C_c for valid cells and a large constant for
// c >= m, so that padding lanes never fall below any cut.
// 24-bit products are exact here: |k|, |na - nr| <= m and the slope is +-2P
// with 2P < 2^21.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "uavq_device.h"

namespace uavq {

namespace {

constexpr int kBigK = 1 << 29;   // K of padding lanes: dE stays far above every cut

// LDS pointers with their address space spelled out, so that offsets stay
// 32-bit (a generic pointer makes the compiler form 64-bit addresses)
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) u32x4 lds_u32x4;

__device__ __forceinline__ bool lane_in_mask(uint32_t lo, uint32_t hi) {
    return __builtin_amdgcn_inverse_ballot_w64(((uint64_t)hi << 32) | (uint64_t)lo);
}

// c + a b with a, b in 24 bits, as one full-rate v_mad_i32_i24 (written out: for a byte a, the
// compiler otherwise picks the 64-bit v_mad_u64_u32 for the product and the add)
__device__ __forceinline__ int mad_i24(int a, int b, int c) {
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

__device__ __forceinline__ uint32_t rl(uint32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
// value v into the lane `lane` of old (one compare shared by the caller's selects)
__device__ __forceinline__ uint32_t wl(uint32_t v, bool mine, uint32_t old) { return mine ? v : old; }

// Step summary R | (q << 16): R set cells and, for p the lowest set cell (0
// if none), q = p m, the offset of its cost row, while that fits 16 bits
// (m <= 256, up to four chunks); q = p for more chunks, multiplied at use.
template <int NJ>
struct Summary {
    static constexpr bool kOffset = NJ <= 4;
    static __device__ __forceinline__ uint32_t key(uint32_t p, int m) {
        return kOffset ? p * (uint32_t)m : p;
    }
    static __device__ __forceinline__ uint32_t row(uint32_t sv, int m) {   // cost-row offset of a summary
        return kOffset ? (sv >> 16) : __umul24(sv >> 16, (uint32_t)m);
    }
};

template <int NJ>
__device__ __forceinline__ uint32_t summary(const uint32_t (&mk)[2 * NJ], int m) {
    uint32_t R = 0, p = 0;
#pragma unroll
    for (int w = 2 * NJ - 1; w >= 0; w--) {
        R += (uint32_t)__popc(mk[w]);
        if (mk[w]) p = 32u * (uint32_t)w + (uint32_t)__builtin_ctz(mk[w]);
    }
    return R | (Summary<NJ>::key(p, m) << 16);   // unsigned: the key may reach bit 31 after the shift
}

}  // namespace

// Where the cost matrix is read from: bytes in LDS, or (DG) 16-bit entries in
// global memory, read through L2 (fields whose matrix does not fit LDS, or
// whose costs exceed a byte; lanes past m read up to 64 kMaxChunks entries
// beyond the matrix, which the plan pads).
template <bool DG>
struct CostSrc {
    typedef const lds_u8 *ptr;
};
template <>
struct CostSrc<true> {
    typedef const uint16_t *ptr;
};

template <int NJ, bool STOP, bool DG = false>
__device__ __forceinline__ void chunk_item(const KArgs &a, int itx, uint8_t *smem) {
    // uint4 chunks of the next table row held in registers during a sweep (none
    // for three chunks: the registers go to the walk; the row is read from L2)
    constexpr int KP = NJ == 2 ? 2 : 0;
    const WorkItem it = a.items[itx];
    const InstDesc d = a.desc[it.inst];
    const int m = d.m, W = d.row_words, twoP = 2 * d.P, fourP = 4 * d.P;
    const int wave = threadIdx.x >> 6, L = threadIdx.x & 63;
    const int nthr = blockDim.x;
    const int Ts = a.thr_stride;
    const int srow = d.sched_row, dstep = d.sched_step;

    // LDS: the acceptance-table row | D (m*m bytes) | start-cell costs (m bytes)
    lds_u8 *const lsm = (lds_u8 *)smem;
    lds_u32 *const sthr = (lds_u32 *)lsm;
    typename CostSrc<DG>::ptr sD, sdep;
    if constexpr (DG) {
        sD = reinterpret_cast<const uint16_t *>(a.ws + d.d_off);
        sdep = reinterpret_cast<const uint16_t *>(a.ws + d.ddep_off);
    } else {
        sD = lsm + 4 * Ts;
        sdep = sD + (int)al16((size_t)m * m);
    }
    // the per-wave words of the last chunk's packed draws (two and three chunks, costs in LDS, when the launch
    // gives the 1 KB per wave): 64 lanes x uint4
    constexpr bool kPW = NJ <= 3 && !DG;
    lds_u32 *const pwd = (lds_u32 *)(lsm + 4 * Ts + (DG ? 16 : (int)(al16((size_t)m * m) + al16((size_t)m) + 64)) +
                                     1024 * wave);
    __shared__ int s_first_sh;
    __shared__ int s_live[2];

    {
        const uint4 *gD = reinterpret_cast<const uint4 *>(a.ws + d.d_off);
        const uint4 *gdep = reinterpret_cast<const uint4 *>(a.ws + d.ddep_off);
        const int nD4 = (m * m + 15) >> 4, nd4 = (m + 15) >> 4;
        uint4 *gsD = reinterpret_cast<uint4 *>(smem + 4 * (size_t)Ts);   // the copies go through generic pointers
        uint4 *gsdep = reinterpret_cast<uint4 *>(smem + 4 * (size_t)Ts + al16((size_t)m * m));
        if (!DG) {
            for (int i = threadIdx.x; i < nD4; i += nthr) gsD[i] = gD[i];
            for (int i = threadIdx.x; i < nd4; i += nthr) gsdep[i] = gdep[i];
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
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        for (int i = threadIdx.x; i < n4; i += nthr) dst[i] = src[i];
    }
    __syncthreads();

    // ---- replica state: lane L holds the cell masks of steps 64 j + L + 1
    uint32_t rm[NJ][2 * NJ];
    uint32_t *st = a.states + d.state_off + (int64_t)r * d.state_words;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int t = 64 * j + L + 1;
#pragma unroll
        for (int w = 0; w < 2 * NJ; w++) rm[j][w] = (active && t <= m && w < W) ? st[(t - 1) * W + w] : 0u;
    }
    if (active && !a.resume) {   // the best state starts as the initial state
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
    // start-cell costs of this lane's cells (the fixed rows 0 and m+1): kept in
    // registers from four chunks on; up to three chunks, where the 1024-thread
    // bound leaves 128 registers, read where needed (fewer spills)
    constexpr bool kDepRegs = NJ >= 4;
    int depr[kDepRegs ? NJ : 1];
#pragma unroll
    for (int j = 0; j < (kDepRegs ? NJ : 1); j++) {
        const int c = 64 * j + L;
        depr[j] = kDepRegs && c < m ? (int)sdep[c] : 0;
    }
    auto dep = [&](int j) -> int {
        if constexpr (kDepRegs) {
            return depr[j];
        } else {
            const int c = 64 * j + L;
            return c < m ? (int)sdep[c] : 0;
        }
    };
    // occupation counts and initial energy (grouped pair sums of the QUBO)
    int Cc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; j++) Cc[j] = 0;
    int64_t E = 0;
    if (active) {
        int64_t lane_e = 0, rowterm = 0;
        int Yp[NJ];
#pragma unroll
        for (int j = 0; j < NJ; j++) Yp[j] = dep(j);
#pragma unroll
        for (int jt = 0; jt < NJ; jt++)
            for (int lt = 0; lt < 64; lt++) {
                const int t = 64 * jt + lt + 1;
                if (t > m) break;
                uint32_t mk[2 * NJ];
#pragma unroll
                for (int w = 0; w < 2 * NJ; w++) mk[w] = rl(rm[jt][w], lt);
                int R = 0;
#pragma unroll
                for (int w = 0; w < 2 * NJ; w++) R += __popc(mk[w]);
                rowterm += (int64_t)d.P * R * (R - 1) - (int64_t)twoP * R;
                int Yt[NJ];
#pragma unroll
                for (int j = 0; j < NJ; j++) {
                    const int x = lane_in_mask(mk[2 * j], mk[2 * j + 1]) ? 1 : 0;
                    Cc[j] += x;
                    lane_e += x * Yp[j];
                    if (t == m && d.closed && 64 * j + L < m) lane_e += x * dep(j);
                    Yt[j] = 0;
                }
#pragma unroll
                for (int w = 0; w < 2 * NJ; w++) {
                    uint32_t bits = mk[w];
                    while (bits) {
                        const int b = __builtin_ctz(bits);
                        bits &= bits - 1u;
                        const auto row = sD + __umul24(32 * w + b, m);   // 24-bit product: one full-rate multiply-add
#pragma unroll
                        for (int j = 0; j < NJ; j++) Yt[j] += row[64 * j + L];
                    }
                }
#pragma unroll
                for (int j = 0; j < NJ; j++) Yp[j] = Yt[j];
            }
#pragma unroll
        for (int j = 0; j < NJ; j++)
            if (64 * j + L < m) lane_e += (int64_t)d.P * Cc[j] * (Cc[j] - 1);
        E = d.c0 + rowterm + wave_sum64(lane_e);
    }
    int KC[NJ];    // 2P C_c; padding lanes far above every cut
    uint32_t si[NJ];    // step summaries of steps 64 j + L + 1
    uint32_t ckey[NJ];  // the summary of a step that holds exactly this lane's cell
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        KC[j] = 64 * j + L < m ? twoP * Cc[j] : kBigK;
        si[j] = summary<NJ>(rm[j], m);
        ckey[j] = (Summary<NJ>::key((uint32_t)(64 * j + L), m) << 16) | 1u;
    }

    int64_t bestE = LLONG_MAX;
    int bestS = -1;
    uint64_t nacc = 0, ndraw = 0;
    if (active && a.resume) {
        bestE = a.best_E[grep];
        bestS = a.best_sweep[grep];
    }
    int64_t Elane = 0;         // energy change of the lane's accepted flips in the current sweep
    bool frozen = false;

    // travel row of step t (uniform) for this lane's cells: the start-cell costs
    // at t = m + 1 (closed tour), 0 past it; from the summary when the step holds
    // one cell, from its mask otherwise.  q = the step's lane in chunk jq.
    auto yrow = [&](int t, uint32_t sv, const uint32_t *mkq, int (&Y)[NJ]) {
        if (t > m) {
#pragma unroll
            for (int j = 0; j < NJ; j++) Y[j] = (t == m + 1 && d.closed) ? dep(j) : 0;
            return;
        }
        const uint32_t R = sv & 0xffffu;
        if (R == 1) {
            // lanes past m read bytes beyond the row (inside the LDS allocation); unused
            const auto row = sD + Summary<NJ>::row(sv, m);
#pragma unroll
            for (int j = 0; j < NJ; j++) Y[j] = row[64 * j + L];
            return;
        }
#pragma unroll
        for (int j = 0; j < NJ; j++) Y[j] = 0;
        if (R == 0) return;
#pragma unroll
        for (int w = 0; w < 2 * NJ; w++) {
            uint32_t bits = mkq[w];
            while (bits) {
                const int b = __builtin_ctz(bits);
                bits &= bits - 1u;
                const auto row = sD + __umul24(32 * w + b, m);   // 24-bit product: one full-rate multiply-add
#pragma unroll
                for (int j = 0; j < NJ; j++) Y[j] += row[64 * j + L];
            }
        }
    };

    // The last chunk's cells fill only nl = m - 64 (NJ - 1) lanes.  When kp = 64 / nl >= 2 of its blocks fit
    // one wave, hot blocks draw the words and cuts of kp consecutive blocks of that chunk in one Philox call
    // (lane L: block g0 + L / nl, cell 64 (NJ - 1) + L % nl) and fetch each block's from its lanes.
    // (a field of a class taken for its costs alone may leave the last chunk empty: no packing then)
    const int nl = max(m - 64 * (NJ - 1), 1);
    const int kp = m > 64 * (NJ - 1) ? 64 / nl : 1;
    // L / nl as (L ceil(2^16 / nl)) >> 16: exact for L < 64 (the error stays below 64 / 2^16 < 1 - (nl - 1) / nl)
    const uint32_t nl_inv = (65536u + (uint32_t)nl - 1u) / (uint32_t)nl;

    for (int s = s_first; s < a.s_end; s++) {
        // next table row: loads issued now, stored to LDS after this sweep
        uint4 pre[KP > 0 ? KP : 1];
        const bool has_next = s + 1 < a.s_end;
        const int n4_next = has_next ? (uniform_load(a.dcut, srow + (s + 1) * dstep) + 2 + 3) >> 2 : 0;
        const uint4 *src_next = reinterpret_cast<const uint4 *>(a.thr + (size_t)(srow + (s + 1) * dstep) * Ts);
#pragma unroll
        for (int k = 0; k < KP; k++) {
            const int i = threadIdx.x + k * nthr;
            pre[k] = has_next ? src_next[i < n4_next ? i : 0] : make_uint4(0u, 0u, 0u, 0u);
        }
        const lds_u32 *thr = sthr;
        const int dcut = uniform_load(a.dcut, srow + s * dstep);
        const float tl2 = __builtin_amdgcn_exp2f(d.tl2_a + d.tl2_b * (float)s);   // ~ T_s ln 2
        const float e0 = 32.0f * tl2 - 0.5f, dm1 = (float)(dcut - 1);
        if (STOP && threadIdx.x == 0) s_live[(s + 1) & 1] = 0;
        if (active && s >= s0 && !frozen) {
            uint32_t nacc_s = 0, ndraw_s = 0;
            // window of travel rows Y_{t0-1} .. Y_{t0+4} of the current block
            int Yw[6][NJ];
#pragma unroll
            for (int j = 0; j < NJ; j++) Yw[0][j] = dep(j);
#pragma unroll
            for (int k = 1; k <= 5; k++) {
                uint32_t mk[2 * NJ];
                const uint32_t sv = rl(si[0], k - 1);
                if ((sv & 0xffff) > 1)
#pragma unroll
                    for (int w = 0; w < 2 * NJ; w++) mk[w] = rl(rm[0][w], k - 1);
                yrow(k, sv, mk, Yw[k]);
            }
            bool spec = true;
            // one-cell steps: bit L of tmk[j] is set iff step 64 j + L + 1 holds exactly one cell (steps past m
            // hold none), so that the block tests take a shift and a compare; rebuilt after each walked block
            // (up to seven chunks: at nine, the masks' scalar registers cost more in spills than they save)
            constexpr bool kMask = NJ <= 7;
            uint64_t tmk[NJ];
#pragma unroll
            for (int j = 0; j < NJ; j++) tmk[j] = kMask ? ballot64((si[j] & 0xffffu) == 1u) : 0ull;
            bool eager = false;   // the last walked block drew in every chunk (hot): draw this block's up front
            // The state is a permutation (every step one cell, every cell one step) and dcut <= 2P - 2 w_max:
            // a set site's dE = 4P - (Y_{t-1} + Y_{t+1} + 2P) >= 2P - 2 w_max >= dcut is never below the cut, and
            // its v = Y_{t-1} + Y_{t+1} + 2P >= dcut never passes for a clear site's.  Quiet blocks then need only
            // min v >= dcut.  Cleared for the rest of the sweep by an accepted flip.
            bool perm = false;
            if (kMask && dcut <= twoP - 2 * d.wmax) {
                bool ok = true;
#pragma unroll
                for (int j = 0; j < NJ; j++) ok &= 64 * j + L >= m || (KC[j] == twoP && (si[j] & 0xffffu) == 1u);
                perm = !ballot64(!ok);
            }
            int pk_g0 = INT_MIN / 2;   // first block of the packed last-chunk cuts held in pk0, pk1
            int pw_g0 = INT_MIN / 2;   // first block of the packed last-chunk words held in pwd
            uint32_t pk0 = 0u, pk1 = 0u;
            // exact cuts of block tb of the last chunk (lanes < nl), from the packed draw of its group
            auto packed_cuts = [&](int tb) {
                if (tb >= pk_g0 + kp) {
                    // blocks tb .. tb + kp - 1 of the last chunk, one per group of nl lanes
                    pk_g0 = tb;
                    const int pk_b = (int)(__umul24((uint32_t)L, nl_inv) >> 16), pk_c = L - pk_b * nl;
                    const uint4 u4 = philox(make_uint4((uint32_t)(64 * (NJ - 1) + pk_c) + 65536u * (uint32_t)(tb + pk_b),
                                                       (uint32_t)s, (uint32_t)r, d.inst_id),
                                            a.seed, 0u);
                    int c0, c1, c2, c3;
                    accept_cuts(u4, tl2, e0, dm1, dcut, (const uint32_t *)thr, c0, c1, c2, c3);
                    pk0 = (uint32_t)c0 | ((uint32_t)c1 << 16);
                    pk1 = (uint32_t)c2 | ((uint32_t)c3 << 16);
                }
                // lane L < nl takes lane (tb - pk_g0) nl + L; the other lanes are padding
                const int src = ((tb - pk_g0) * nl + L) << 2;
                return make_uint2((uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)pk0),
                                  (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)pk1));
            };
#pragma unroll
            for (int jt = 0; jt < NJ; jt++) {
                int q0 = 0;
                if (kMask && perm) {
                    // The common case once the state is a permutation: blocks of one-cell steps whose next four
                    // steps (same chunk) hold one cell each too, quiet by the min test.  The window moves on and
                    // nothing else changes (what the general loop below does for them, in fewer steps); the
                    // first other block goes to the general loop.
                    while (q0 <= 52 && ((tmk[jt] >> q0) & 0x1efull) == 0x1efull) {
                        int mv = INT_MAX;
#pragma unroll
                        for (int i = 0; i < 4; i++)
#pragma unroll
                            for (int j = 0; j < NJ; j++) mv = min(mv, Yw[i][j] + Yw[i + 2][j] + KC[j]);
                        if (ballot64(mv < dcut)) break;
#pragma unroll
                        for (int j = 0; j < NJ; j++) {
                            Yw[0][j] = Yw[4][j];
                            Yw[1][j] = Yw[5][j];
                        }
#pragma unroll
                        for (int k = 0; k < 4; k++) {
                            const auto row = sD + Summary<NJ>::row(rl(si[jt], q0 + 5 + k), m);
#pragma unroll
                            for (int j = 0; j < NJ; j++) Yw[2 + k][j] = row[64 * j + L];
                        }
                        q0 += 4;
                    }
                }
                for (; q0 < 64; q0 += 4) {
                    const int t0 = 64 * jt + q0 + 1;
                    if (t0 > m) break;
                    const int tb = (t0 - 1) >> 2;
                    // wave priority: the block's tests and walk are chains of dependent instructions and issue
                    // before other waves' Philox stretches (the eager draws and the draws-only test), which fill
                    // the gaps
                    __builtin_amdgcn_s_setprio(1);
                    uint32_t sx[4];   // summaries of the block's steps
#pragma unroll
                    for (int i = 0; i < 4; i++) sx[i] = rl(si[jt], q0 + i);

                    // ---- quiet-block test (every step of the block holds one cell: the
                    // low halves of the four summaries are all 1)
                    bool done = false;
                    bool tours = spec;
                    if constexpr (kMask) {
                        tours = tours && ((tmk[jt] >> q0) & 0xfull) == 0xfull;
                    } else {
                        const uint32_t s_or = sx[0] | sx[1] | sx[2] | sx[3], s_and = sx[0] & sx[1] & sx[2] & sx[3];
                        tours = tours && t0 + 3 <= m && (s_or & 0xfffe) == 0 && (s_and & 1);
                    }
                    // R_t = 1: dE = v for x = 0 and 4P - v for x = 1, v = Y_{t-1} + Y_{t+1} + 2P C_c;
                    // x = 1 exactly at the lane whose cell the summary names
                    auto dEq = [&](int i, int j) {
                        const int v = Yw[i][j] + Yw[i + 2][j] + KC[j];
                        return ckey[j] == sx[i] ? fourP - v : v;
                    };
                    bool quick = false;
                    if (tours && perm) {
                        int mv = INT_MAX;
#pragma unroll
                        for (int i = 0; i < 4; i++)
#pragma unroll
                            for (int j = 0; j < NJ; j++) mv = min(mv, Yw[i][j] + Yw[i + 2][j] + KC[j]);
                        quick = !ballot64(mv < dcut);
                    }
                    if (quick) {
                        done = true;
                    } else if (tours) {
                        int mn = INT_MAX;
#pragma unroll
                        for (int i = 0; i < 4; i++)
#pragma unroll
                            for (int j = 0; j < NJ; j++) mn = min(mn, dEq(i, j));
                        if (!ballot64(mn < dcut)) {
                            done = true;   // nothing below the cut: every site rejected without a draw
                        } else if (!ballot64(mn <= 0)) {
                            __builtin_amdgcn_s_setprio(0);   // the draws: a long stretch with ample parallel work
                            // only draws: take the chunks' words; finished if none accepts
                            bool acc = false;
                            uint32_t nd = 0;
#pragma unroll
                            for (int j = 0; j < NJ; j++) {
                                int dEb[4];
                                bool need[4];
                                bool any = false;
#pragma unroll
                                for (int i = 0; i < 4; i++) {
                                    dEb[i] = dEq(i, j);
                                    need[i] = (uint32_t)(dEb[i] - 1) < (uint32_t)(dcut - 1);
                                    any |= need[i];
                                }
                                if (!ballot64(any)) continue;
                                uint4 u4;
                                if (kPW && a.pw && j == NJ - 1 && kp > 1) {
                                    // the last chunk: one Philox call draws the words of kp consecutive blocks
                                    // (lane L: block g0 + L / nl, cell 64 (NJ - 1) + L % nl), kept in the
                                    // wave's LDS area; block tb takes its lanes' words from there
                                    if (tb >= pw_g0 + kp) {
                                        pw_g0 = tb;
                                        const int pk_b = (int)(__umul24((uint32_t)L, nl_inv) >> 16), pk_c = L - pk_b * nl;
                                        const uint4 w4 = philox(
                                            make_uint4((uint32_t)(64 * (NJ - 1) + pk_c) + 65536u * (uint32_t)(tb + pk_b),
                                                       (uint32_t)s, (uint32_t)r, d.inst_id),
                                            a.seed, 0u);
                                        *(lds_u32x4 *)(pwd + 4 * L) = u32x4{w4.x, w4.y, w4.z, w4.w};
                                    }
                                    const int src = L < nl ? (tb - pw_g0) * nl + L : 0;   // other lanes: padding
                                    const u32x4 w4 = *(const lds_u32x4 *)(pwd + 4 * src);
                                    u4 = make_uint4(w4.x, w4.y, w4.z, w4.w);
                                } else {
                                    u4 = philox(make_uint4((uint32_t)(64 * j + L) + 65536u * (uint32_t)tb, (uint32_t)s,
                                                           (uint32_t)r, d.inst_id),
                                                a.seed, 0u);
                                }
                                const uint32_t uw[4] = {u4.x, u4.y, u4.z, u4.w};
                                // unconditional reads (index 0 where no draw happens) issue together
                                uint32_t th[4];
#pragma unroll
                                for (int i = 0; i < 4; i++) th[i] = thr[need[i] ? dEb[i] : 0];
#pragma unroll
                                for (int i = 0; i < 4; i++) {
                                    acc |= need[i] & (uw[i] < th[i]);
                                    nd += (uint32_t)__popcll(ballot64(need[i]));
                                }
                            }
                            if (!ballot64(acc)) {
                                done = true;
                                ndraw_s += nd;
                            }
                        }
                    }

                    if (!done) {
                        // ---- the block walked step by step (cf. the generic chunked kernel)
                        const uint32_t acc_before = nacc_s;
                        uint32_t have_cut = 0;   // bit j: chunk j's cuts of this block are known
                        uint32_t cutp[NJ][2];
                        if (eager) {
                            __builtin_amdgcn_s_setprio(0);   // a long stretch with ample parallel work
                            // every chunk is likely to need its words: draw them all here, in one
                            // branch-free stretch (the cuts depend on the words and the table only)
#pragma unroll
                            for (int j = 0; j < NJ; j++) {
                                if (j == NJ - 1 && kp > 1) {
                                    const uint2 cw = packed_cuts(tb);
                                    cutp[j][0] = cw.x;
                                    cutp[j][1] = cw.y;
                                    continue;
                                }
                                const uint4 u4 = philox(
                                    make_uint4((uint32_t)(64 * j + L) + 65536u * (uint32_t)tb, (uint32_t)s, (uint32_t)r,
                                               d.inst_id),
                                    a.seed, 0u);
                                int c0, c1, c2, c3;
                                accept_cuts(u4, tl2, e0, dm1, dcut, (const uint32_t *)thr, c0, c1, c2, c3);
                                cutp[j][0] = (uint32_t)c0 | ((uint32_t)c1 << 16);
                                cutp[j][1] = (uint32_t)c2 | ((uint32_t)c3 << 16);
                            }
                            have_cut = (1u << NJ) - 1u;
                        }
                        uint32_t drawn = 0;   // bit j: a site of chunk j needed a draw in this block
                        // the walk is a chain of dependent ballots: it issues first on its SIMD, and the other
                        // waves' Philox stretches fill the gaps
                        __builtin_amdgcn_s_setprio(2);
#pragma unroll
                        for (int i = 0; i < 4; i++) {
                            const int t = t0 + i;
                            if (t > m) break;
                            const int lt = q0 + i;
                            uint32_t mc[2 * NJ];
#pragma unroll
                            for (int w = 0; w < 2 * NJ; w++) mc[w] = rl(rm[jt][w], lt);
                            const int hR1 = twoP * ((int)(sx[i] & 0xffffu) - 1);   // 2P (R_t - 1)
                            int dE0[NJ], dpl[NJ];
                            bool xb[NJ];
#pragma unroll
                            for (int j = 0; j < NJ; j++) {
                                xb[j] = lane_in_mask(mc[2 * j], mc[2 * j + 1]);
                                const int v = Yw[i][j] + Yw[i + 2][j] + KC[j] + hR1;
                                dE0[j] = xb[j] ? fourP - v : v;
                                dpl[j] = xb[j] ? -twoP : twoP;   // change of dE per net 1 gained by step t
                            }
                            int mnv = dE0[0];
#pragma unroll
                            for (int j = 1; j < NJ; j++) mnv = min(mnv, dE0[j]);
                            // a step with no site below the cut is finished: no accept, no draw
                            if (!ballot64(mnv < dcut)) continue;
                            const int ti = i;
                            int k = 0, sg = 1;   // sg: +1 while the pending cost row adds, -1 when it subtracts
                            uint64_t accd[NJ];
                            int dY[NJ], pd[NJ];
#pragma unroll
                            for (int j = 0; j < NJ; j++) {
                                accd[j] = 0;
                                dY[j] = 0;
                                pd[j] = 0;
                            }
                            // flip the first accepted site of chunk j's mask am; its cost-row
                            // entries are read now and added (or subtracted) at the next flip
                            auto flip = [&](int j, uint64_t am, uint64_t &openm) {
                                const int Ls = __builtin_ctzll(am);
                                accd[j] |= 1ull << Ls;
                                const uint64_t rowj = ((uint64_t)mc[2 * j + 1] << 32) | (uint64_t)mc[2 * j];
                                const bool clears = (rowj >> Ls) & 1ull;
#pragma unroll
                                for (int jj = 0; jj < NJ; jj++) dY[jj] = mad_i24(pd[jj], sg, dY[jj]);
                                const auto drow = sD + (64 * j + Ls) * m;
#pragma unroll
                                for (int jj = 0; jj < NJ; jj++) pd[jj] = drow[64 * jj + L];
                                sg = clears ? -1 : 1;
                                k += clears ? -1 : 1;
                                openm &= ~1ull << Ls;   // the walk resumes after Ls
                            };
#pragma unroll
                            for (int j = 0; j < NJ; j++) {
                                if (64 * j >= m) break;
                                uint64_t openm = m - 64 * j >= 64 ? ~0ull : ((1ull << (m - 64 * j)) - 1ull);
                                bool walking = true;
                                if (!((have_cut >> j) & 1u)) {
                                    // no exact cut yet: accept iff dE <= 0 while no open site of the
                                    // chunk needs a draw; then the chunk's words and cuts are drawn
                                    while (true) {
                                        const int dE = dE0[j] + __mul24(k, dpl[j]);
                                        if (ballot64((uint32_t)(dE - 1) < (uint32_t)(dcut - 1)) & openm) {
                                            have_cut |= 1u << j;
                                            const uint2 cw = draw_cuts((uint32_t)(64 * j + L) + 65536u * (uint32_t)tb,
                                                                       (uint32_t)s, (uint32_t)r, d.inst_id, a.seed, tl2,
                                                                       e0, dm1, dcut, (const uint32_t *)thr);
                                            cutp[j][0] = cw.x;
                                            cutp[j][1] = cw.y;
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
                                    const int rel = cut - dE0[j];   // accept iff k dpl < cut - dE0
                                    uint64_t am = ballot64(__mul24(k, dpl[j]) < rel) & openm;
                                    while (am) {
                                        flip(j, am, openm);
                                        am = ballot64(__mul24(k, dpl[j]) < rel) & openm;
                                    }
                                }
                            }
                            bool any = false;
#pragma unroll
                            for (int j = 0; j < NJ; j++) any |= accd[j] != 0;
                            if (!any) {
                                // no flip: every site was visited with its dE0
#pragma unroll
                                for (int j = 0; j < NJ; j++) {
                                    const uint32_t nd = (uint32_t)__popcll(
                                        ballot64((uint32_t)(dE0[j] - 1) < (uint32_t)(dcut - 1)));
                                    ndraw_s += nd;
                                    drawn |= nd ? 1u << j : 0u;
                                }
                            } else {
#pragma unroll
                                for (int jj = 0; jj < NJ; jj++) dY[jj] = mad_i24(pd[jj], sg, dY[jj]);
                                // visit-time dE of every site (dE0 plus the slope per net flip
                                // before it in site order), then draws, energy, counts and masks
                                int nab = 0, nrb = 0;   // adds / removes in earlier chunks
#pragma unroll
                                for (int j = 0; j < NJ; j++) {
                                    if (!accd[j]) {
                                        // no flip in this chunk: every site saw dE0 plus the earlier chunks' net flips
                                        const int dEv = dE0[j] + __mul24(nab - nrb, dpl[j]);
                                        const uint32_t nd = (uint32_t)__popcll(
                                            ballot64((uint32_t)(dEv - 1) < (uint32_t)(dcut - 1)));
                                        ndraw_s += nd;
                                        drawn |= nd ? 1u << j : 0u;
                                        Yw[i + 1][j] += dY[j];
                                        continue;
                                    }
                                    const uint64_t rowj = ((uint64_t)mc[2 * j + 1] << 32) | (uint64_t)mc[2 * j];
                                    const uint64_t adds = accd[j] & ~rowj, rems = accd[j] & rowj;
                                    const int na = nab + (int)__builtin_amdgcn_mbcnt_hi(
                                                             (uint32_t)(adds >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)adds, 0u));
                                    const int nr = nrb + (int)__builtin_amdgcn_mbcnt_hi(
                                                             (uint32_t)(rems >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)rems, 0u));
                                    const int dEv = dE0[j] + __mul24(na - nr, dpl[j]);
                                    const uint32_t nd =
                                        (uint32_t)__popcll(ballot64((uint32_t)(dEv - 1) < (uint32_t)(dcut - 1)));
                                    ndraw_s += nd;
                                    drawn |= nd ? 1u << j : 0u;
                                    const bool inA = lane_in_mask((uint32_t)accd[j], (uint32_t)(accd[j] >> 32));
                                    Elane += inA ? dEv : 0;
                                    KC[j] += inA ? dpl[j] : 0;
                                    Yw[i + 1][j] += dY[j];
                                    nab += (int)__popcll(adds);
                                    nrb += (int)__popcll(rems);
                                    nacc_s += (uint32_t)__popcll(accd[j]);
                                }
#pragma unroll
                                for (int j = 0; j < NJ; j++) {
                                    mc[2 * j] ^= (uint32_t)accd[j];
                                    mc[2 * j + 1] ^= (uint32_t)(accd[j] >> 32);
                                }
                                const bool mine = L == lt;
#pragma unroll
                                for (int w = 0; w < 2 * NJ; w++) rm[jt][w] = wl(mc[w], mine, rm[jt][w]);
                                si[jt] = wl(summary<NJ>(mc, m), mine, si[jt]);
                            }
                        }
                        spec = nacc_s == acc_before;
                        perm = perm && spec;
                        eager = drawn == (1u << NJ) - 1u && !spec;
                        __builtin_amdgcn_s_setprio(0);
                        // the masks again from the summaries (not held over the walk, whose registers are scarce)
#pragma unroll
                        for (int j = 0; j < NJ; j++) tmk[j] = kMask ? ballot64((si[j] & 0xffffu) == 1u) : 0ull;
                    }
                    // shift the window by four steps; the new rows (steps t0+5 .. t0+8:
                    // lanes q0+5.. of chunk jt, or of chunk jt+1 past lane 63) were not
                    // touched by this block's walk
#pragma unroll
                    for (int j = 0; j < NJ; j++) {
                        Yw[0][j] = Yw[4][j];
                        Yw[1][j] = Yw[5][j];
                    }
                    {
                        uint32_t sv[4];
                        if (q0 <= 52 || jt + 1 >= NJ) {
#pragma unroll
                            for (int k = 0; k < 4; k++) sv[k] = rl(si[jt], min(q0 + 5 + k, 63));   // past 63: t > m
                        } else {
#pragma unroll
                            for (int k = 0; k < 4; k++) {
                                const int q = q0 + 5 + k;
                                sv[k] = q < 64 ? rl(si[jt], q) : rl(si[jt + 1 < NJ ? jt + 1 : jt], q - 64);
                            }
                        }
                        // steps t0+5 .. t0+8 are lanes q0+5 .. q0+8 of chunk jt, past 63 of chunk jt + 1
                        bool ntours;
                        if constexpr (kMask) {
                            const int sh = q0 + 5;   // 5 .. 65
                            uint64_t nb = sh < 64 ? tmk[jt] >> sh : 0ull;
                            if (jt + 1 < NJ && sh > 60) {
                                const uint64_t hi = tmk[jt + 1 < NJ ? jt + 1 : jt];
                                nb = sh < 64 ? nb | (hi << (64 - sh)) : hi >> (sh - 64);
                            }
                            ntours = (nb & 0xfull) == 0xfull;
                        } else {
                            const uint32_t l_or = sv[0] | sv[1] | sv[2] | sv[3], l_and = sv[0] & sv[1] & sv[2] & sv[3];
                            ntours = t0 + 8 <= m && (l_or & 0xfffe) == 0 && (l_and & 1);
                        }
                        if (ntours) {
                            // four one-cell steps: their cost rows
#pragma unroll
                            for (int k = 0; k < 4; k++) {
                                const auto row = sD + Summary<NJ>::row(sv[k], m);
#pragma unroll
                                for (int j = 0; j < NJ; j++) Yw[2 + k][j] = row[64 * j + L];
                            }
                        } else {
#pragma unroll
                            for (int k = 0; k < 4; k++) {
                                const int q = q0 + 5 + k, t = t0 + 5 + k;
                                uint32_t mk[2 * NJ];
                                if (t <= m && (sv[k] & 0xffff) > 1) {
                                    if (q < 64 || jt + 1 >= NJ) {
#pragma unroll
                                        for (int w = 0; w < 2 * NJ; w++) mk[w] = rl(rm[jt][w], q & 63);
                                    } else {
#pragma unroll
                                        for (int w = 0; w < 2 * NJ; w++)
                                            mk[w] = rl(rm[jt + 1 < NJ ? jt + 1 : jt][w], q - 64);
                                    }
                                }
                                yrow(t, sv[k], mk, Yw[2 + k]);
                            }
                        }
                    }
                }
            }
            nacc += nacc_s;
            ndraw += ndraw_s;
            if (STOP && nacc_s == 0 && ndraw_s == 0) frozen = true;
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
        if (STOP && L == 0 && active && !frozen) atomicAdd(&s_live[s & 1], 1);
        // one table row in LDS: every wave is done with row s before row s + 1 replaces it
        __syncthreads();
        const bool all_frozen = STOP && s_live[s & 1] == 0;
        if (has_next) {
            uint4 *dst = reinterpret_cast<uint4 *>(smem);
#pragma unroll
            for (int k = 0; k < KP; k++) {
                const int i = threadIdx.x + k * nthr;
                if (i < n4_next) dst[i] = pre[k];
            }
            for (int i = threadIdx.x + KP * nthr; i < n4_next; i += nthr) dst[i] = src_next[i];
        }
        __syncthreads();
        if (all_frozen) break;
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
